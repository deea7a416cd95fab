"""The commutation rule behind the tile passes' look-ahead, pinned on the
FP64 oracle (no GPU).

A tile pass may take a later step ahead of steps it leaves behind when the
two commute: neither mixes a qubit the other touches (a window mixes its
measured qubit into the new one; an E or Z only reads signs), and they are
not two windows whose probability depends on the state (an even number of
E between the measured and the new qubit).  A window with an odd count has
p = 1/2 for every state (Eqs. 11-13) and acts as a unitary times a fixed
factor, so the probabilities of the steps around it do not depend on the
order.  Here whole gate chunks of a pattern (a window N w; E...; M v; X w,
or a CZ) are swapped at random where the rule allows it; the oracle's
output and every measurement's probability are unchanged.  Swapping two
windows with an even count (which the rule forbids) changes the recorded
probabilities, so that part of the rule is needed.
"""
import math

import numpy as np

import owqs_workloads as W
from oracle import core as oc


def chunks_of(n_logical, g, n_gates, even_share):
    """Gate chunks on n_logical wires: windows (E(v, w) once, or twice with
    probability even_share) and CZs; each chunk records the qubits it
    touches, whether it is a window and whether its E(v, w) count is even."""
    cur = list(range(n_logical))
    nxt = n_logical
    out = []
    for _ in range(n_gates):
        if g.random() < 0.8:
            q = int(g.integers(n_logical))
            u, w = cur[q], nxt
            nxt += 1
            even = bool(g.random() < even_share)
            cmds = [("N", w), ("E", u, w)] + ([("E", u, w)] if even else []) + \
                   [("M", u, float(g.uniform(0, 2 * math.pi)), (), ()), ("X", w, (u,))]
            out.append({"cmds": cmds, "touch": {u, w}, "window": True, "even": even, "m": u})
            cur[q] = w
        else:
            a, b = (int(x) for x in g.choice(n_logical, size=2, replace=False))
            out.append({"cmds": [("E", cur[a], cur[b])], "touch": {cur[a], cur[b]}, "window": False,
                        "even": False, "m": None})
    return out, cur


def may_swap(a, b):
    if a["touch"] & b["touch"]:
        return False
    return not (a["window"] and b["window"] and a["even"] and b["even"])


def run_chunks(chunks, n_logical, outputs, outcome_of, inp):
    cmds = [c for ch in chunks for c in ch["cmds"]]
    pat = W.Pattern(list(range(n_logical)), outputs, cmds)
    meas = [c[1] for c in cmds if c[0] == "M"]
    psi, probs = oc.run(pat, [outcome_of[q] for q in meas], inp)
    return psi, dict(zip(meas, probs))


def test_swaps_allowed_by_the_rule_keep_output_and_probabilities():
    for seed in range(6):
        g = np.random.default_rng(7000 + seed)
        n = 5
        chunks, outputs = chunks_of(n, g, 40, even_share=0.3)
        outcome_of = {ch["m"]: int(g.integers(2)) for ch in chunks if ch["window"]}
        inp = W.gaussian_state(n, g).astype(np.complex128)
        inp /= np.linalg.norm(inp)  # in FP64: the first M's p would carry the complex64 norm error
        psi0, p0 = run_chunks(chunks, n, outputs, outcome_of, inp)
        order = list(chunks)
        swaps = 0
        for _ in range(400):
            i = int(g.integers(len(order) - 1))
            if may_swap(order[i], order[i + 1]):
                order[i], order[i + 1] = order[i + 1], order[i]
                swaps += 1
        assert swaps > 50
        psi1, p1 = run_chunks(order, n, outputs, outcome_of, inp)
        assert np.max(np.abs(psi1 - psi0)) <= 1e-12, seed
        for q in p0:
            assert abs(p1[q] - p0[q]) <= 1e-12, (seed, q)


def test_two_even_windows_do_not_swap_freely():
    """Two windows with an even E(v, w) count on different wires commute as
    operators (the output is the same), but each records a conditional
    probability that depends on which was measured first."""
    worst = 0.0
    for seed in range(20):
        g = np.random.default_rng(7100 + seed)
        n = 3
        inp = W.gaussian_state(n, g).astype(np.complex128)
        inp /= np.linalg.norm(inp)
        # entangle the wires first, so that the two measurements correlate
        pre = [{"cmds": [("E", 0, 1)], "touch": {0, 1}, "window": False, "even": False, "m": None},
               {"cmds": [("E", 1, 2)], "touch": {1, 2}, "window": False, "even": False, "m": None}]
        a = {"cmds": [("N", 3), ("E", 0, 3), ("E", 0, 3), ("M", 0, float(g.uniform(0, 6.28)), (), ()),
                      ("X", 3, (0,))], "touch": {0, 3}, "window": True, "even": True, "m": 0}
        b = {"cmds": [("N", 4), ("E", 2, 4), ("E", 2, 4), ("M", 2, float(g.uniform(0, 6.28)), (), ()),
                      ("X", 4, (2,))], "touch": {2, 4}, "window": True, "even": True, "m": 2}
        assert not may_swap(a, b)
        outcome_of = {0: int(g.integers(2)), 2: int(g.integers(2))}
        psi_ab, p_ab = run_chunks(pre + [a, b], n, [3, 1, 4], outcome_of, inp)
        psi_ba, p_ba = run_chunks(pre + [b, a], n, [3, 1, 4], outcome_of, inp)
        assert np.max(np.abs(psi_ab - psi_ba)) <= 1e-12
        worst = max(worst, abs(p_ab[0] - p_ba[0]), abs(p_ab[2] - p_ba[2]))
    assert worst > 1e-3
