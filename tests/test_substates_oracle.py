"""Pins of the sub-state oracle (Sec. 4.1, Sec. 4.4.1) on the CPU: Fig. 8's
printed sub-states at every stage, the sub-state partition against the
connected components of the applied E's, the assembled state against the
elimination oracle, and the sub-state widths at each M against the
reordering oracle's state-spaces (Table I)."""
import json
import math
import os

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc
from oracle import proa
from oracle import substates as so

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SQ2 = math.sqrt(2.0)


def _den(s):
    return {"1": 1.0, "2": 2.0, "sqrt2": SQ2, "2sqrt2": 2 * SQ2}[s]


def test_fig8_substates_stage_by_stage():
    """Fig. 8 (Sec. 4.7): the CNOT pattern of Eq. 23 on |q2 q1> = |11> as two
    one-qubit input sub-states; after each printed stage the sub-states (which
    qubits, and their amplitudes) are the printed ones."""
    gold = json.load(open(os.path.join(GOLD, "fig8_cnot.json")))
    cmds = [("N", 3), ("N", 4), ("E", 2, 3), ("M", 2, 0.0, (), ()), ("E", 3, 4), ("E", 1, 3),
            ("M", 3, 0.0, (), ()), ("Z", 1, (2,)), ("Z", 4, (2,)), ("X", 4, (3,))]
    pat = W.Pattern([1, 2], [1, 4], cmds)
    factors = [([1], np.array([0, 1.0])), ([2], np.array([0, 1.0]))]
    stops = {"a": 2, "b": 3, "c": 4, "d": 6, "e": 7, "f": len(cmds)}
    for stage in gold["stages"]:
        st, _ = so.run(pat, [0, 1], factors, stop=stops[stage["label"]])
        want = {tuple(sorted(s["qubits"])): s for s in stage["substates"]}
        got = {tuple(sorted(qs)): (qs, vec) for qs, vec in st.subs}
        assert set(got) == set(want), stage["label"]
        for key, s in want.items():
            qs, vec = got[key]
            printed = np.array(s["num"], np.complex128) / _den(s["den"])
            # printed kets list the most significant qubit first
            np.testing.assert_allclose(so.factor_in_order(qs, vec, s["qubits"][::-1]), printed, atol=1e-14,
                                       err_msg=stage["label"])
        assert abs(st.scalar - 1.0) < 1e-14


def _components(pattern, stop, live):
    """Connected components of the qubits touched so far under the applied E's
    (measured qubits still connect), restricted to the live qubits."""
    parent = {}

    def find(x):
        parent.setdefault(x, x)
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    ins = list(pattern.inputs)
    for q in ins:
        find(q)
    for a, b in zip(ins, ins[1:]):
        parent[find(a)] = find(b)
    for c in pattern.cmds[:stop]:
        find(c[1])
        if c[0] == "E":
            parent[find(c[1])] = find(c[2])
    groups = {}
    for q in live:
        groups.setdefault(find(q), []).append(q)
    return sorted(sorted(g) for g in groups.values())


def test_partition_is_the_components_of_the_applied_e():
    g = np.random.default_rng(4601)
    for i in range(30):
        pat = W.random_pattern(g)
        per = [int(b) for b in g.integers(0, 2, pat.n_meas())]
        inp = W.gaussian_state(len(pat.inputs), g).astype(np.complex128)
        factors = [(list(pat.inputs), inp)] if pat.inputs else None
        for stop in range(0, len(pat.cmds) + 1, max(1, len(pat.cmds) // 6)):
            try:
                st, _ = so.run(pat, per, factors, stop=stop)
            except so.SubStateError:
                break   # a forced outcome of probability 0
            live = [q for qs in st.partition() for q in qs]
            assert sorted(sorted(p) for p in st.partition()) == _components(pat, stop, live)


@pytest.mark.parametrize("mode", [so.MODE_OWQS, so.MODE_EOWQS])
def test_assembled_state_equals_the_elimination_oracle(mode):
    g = np.random.default_rng(4602 + mode)
    done = 0
    for attempt in range(200):
        if mode == so.MODE_OWQS:
            pat = W.random_pattern(g)
        else:  # EOWQS needs p = 1/2: flow patterns of J/CZ circuits
            nl = int(g.integers(1, 5))
            pat = W.circuit_to_pattern(nl, W.random_jcz_circuit(nl, int(g.integers(1, 12)), int(g.integers(0, 4)) if nl > 1 else 0, g))
        per = [int(b) for b in g.integers(0, 2, pat.n_meas())]
        inp = W.gaussian_state(len(pat.inputs), g).astype(np.complex128) if pat.inputs else None
        try:
            want, pw = oc.run(pat, per, inp, mode=mode)
        except oc.OracleError:
            continue
        st, pg = so.run(pat, per, [(list(pat.inputs), inp)] if pat.inputs else None, mode=mode)
        np.testing.assert_allclose(so.assemble(st, pat.outputs), want, atol=1e-12)
        np.testing.assert_allclose(pg, pw, atol=1e-12)
        assert st.widest <= max(pat.max_live(), 1)
        done += 1
    assert done >= 30


def test_separate_components_stay_separate():
    """Two J/CZ circuits on disjoint qubits, interleaved: never more than one
    circuit's width in one sub-state, and the result is the product."""
    g = np.random.default_rng(4603)
    ga = W.random_jcz_circuit(3, 12, 3, g)
    gb = W.random_jcz_circuit(3, 12, 3, g)
    pa = W.circuit_to_pattern(3, ga)
    pb = W.circuit_to_pattern(3, gb)
    off = 1000
    shift = lambda c: (c[0],) + tuple((x + off if isinstance(x, (int, np.integer)) else
                                        tuple(y + off for y in x) if isinstance(x, tuple) else x)
                                       for x in c[1:])
    cb = [shift(c) if c[0] != "M" else ("M", c[1] + off, c[2], tuple(y + off for y in c[3]),
                                         tuple(y + off for y in c[4])) for c in pb.cmds]
    cmds = []
    for k in range(max(len(pa.cmds), len(cb))):
        if k < len(pa.cmds):
            cmds.append(pa.cmds[k])
        if k < len(cb):
            cmds.append(cb[k])
    both = W.Pattern(list(pa.inputs) + [q + off for q in pb.inputs], list(pa.outputs) + [q + off for q in pb.outputs],
                     cmds)
    ia = W.gaussian_state(3, g).astype(np.complex128)
    ib = W.gaussian_state(3, g).astype(np.complex128)
    st, _ = so.run(both, np.zeros(both.n_meas(), np.uint8),
                   [(list(pa.inputs), ia), ([q + off for q in pb.inputs], ib)], mode=so.MODE_EOWQS)
    assert st.widest <= max(pa.max_live(), pb.max_live())
    assert len(st.subs) == 2
    wa, _ = oc.run(pa, np.zeros(pa.n_meas(), np.uint8), ia, mode=oc.MODE_EOWQS)
    wb, _ = oc.run(pb, np.zeros(pb.n_meas(), np.uint8), ib, mode=oc.MODE_EOWQS)
    np.testing.assert_allclose(so.assemble(st, both.outputs), np.kron(wb, wa), atol=1e-12)


def test_widths_at_measurement_are_the_proa_state_spaces():
    """Run in PROA's order, the measured qubit's sub-state is MS(v) (Sec. 4.3):
    Table I's state-space sizes, and the same on random standard patterns."""
    gold = json.load(open(os.path.join(GOLD, "table1_swap_proa.json")))
    cmds = [("N", q) for q in gold["qubits"]] + [("E", a, b) for a, b in gold["edges"]]
    cmds += [("M", q, 0.0, (), ()) for q in gold["qubits"] if q not in gold["outputs"]]
    pat = W.Pattern([], gold["outputs"], cmds)
    re = proa.reordered_pattern(pat, gold["order"])
    st, _ = so.run(re, np.zeros(re.n_meas(), np.uint8), mode=so.MODE_EOWQS)
    assert st.at_measure == [len(s) for s in gold["measurement_state_spaces"]]
    g = np.random.default_rng(4604)
    for _ in range(20):
        pat = W.random_standard_pattern(g, n_qubits=int(g.integers(5, 12)), n_in=0, n_out=int(g.integers(1, 3)),
                                        extra_edges=int(g.integers(0, 5)))
        order, spaces, m, _ = proa.proa(pat)
        re = proa.reordered_pattern(pat, order)
        st, _ = so.run(re, np.zeros(re.n_meas(), np.uint8), mode=so.MODE_EOWQS)
        assert st.at_measure == [len(s) for s in spaces]
