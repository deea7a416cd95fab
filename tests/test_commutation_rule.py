"""The commutation rule behind the tile passes' look-ahead, pinned on the
FP64 oracle (no GPU).

A tile pass may take a later step ahead of steps it leaves behind when the
two commute: neither mixes a wire (a window mixes its measured qubit into
the new one on the same wire; an X swaps pairs) that the other mixes or
reads as a sign (an E or a Z, a window's E partners), and they are not two
windows whose probability depends on the state (an even number of E
between the measured and the new qubit).  Steps that only read a wire as a
sign may share it.  A window with an odd count has p = 1/2 for every state
(Eqs. 11-13) and acts as a unitary times a fixed factor, so the
probabilities of the steps around it do not depend on the order.  Here
whole chunks of a pattern (a window N w; E...; M v; X w with E partners on
other wires, a CZ, an X or Z correction) are swapped at random where the
rule allows it; the oracle's output and every measurement's probability
are unchanged.  Pairs that the rule keeps apart change the output when
swapped, and swapping two windows with an even count (which the rule
forbids) changes the recorded probabilities, so each part of the rule is
needed.
"""
import math

import numpy as np

import owqs_workloads as W
from oracle import core as oc


def chunks_of(n_logical, g, n_gates, even_share, signal_qubit):
    """Gate chunks on n_logical wires, each with the wires it mixes and the
    wires it reads as signs, as the host's grouping sees them:

    * a window on wire q (N w; E(v, w) once, or twice with probability
      even_share; E(v, x) to other wires, whose bits become sign masks;
      M v; X w) mixes q and reads its E partners as signs;
    * a CZ on wires a, b reads both as signs;
    * an X correction on wire q mixes q, a Z correction reads q as a sign
      (both with the signal of `signal_qubit`, measured before every chunk).
    """
    cur = list(range(n_logical))
    nxt = n_logical + 1
    out = []
    for _ in range(n_gates):
        r = g.random()
        if r < 0.6:
            q = int(g.integers(n_logical))
            u, w = cur[q], nxt
            nxt += 1
            even = bool(g.random() < even_share)
            others = [x for x in range(n_logical) if x != q and g.random() < 0.25]
            cmds = [("N", w), ("E", u, w)] + ([("E", u, w)] if even else []) + \
                   [("E", u, cur[x]) for x in others] + \
                   [("M", u, float(g.uniform(0, 2 * math.pi)), (), ()), ("X", w, (u,))]
            out.append({"cmds": cmds, "mix": {q}, "diag": set(others), "window": True, "even": even, "m": u})
            cur[q] = w
        elif r < 0.8:
            a, b = (int(x) for x in g.choice(n_logical, size=2, replace=False))
            out.append({"cmds": [("E", cur[a], cur[b])], "mix": set(), "diag": {a, b}, "window": False,
                        "even": False, "m": None})
        else:
            q = int(g.integers(n_logical))
            op = "X" if g.random() < 0.5 else "Z"
            out.append({"cmds": [(op, cur[q], (signal_qubit,))], "mix": {q} if op == "X" else set(),
                        "diag": {q} if op == "Z" else set(), "window": False, "even": False, "m": None})
    return out, cur


def may_swap(a, b):
    """The host's rule (commute_steps): neither mixes a wire that the other
    mixes or reads as a sign, and not two windows with an even E(v, w)
    count.  Steps that only read a wire as a sign may share it."""
    if a["mix"] & (b["mix"] | b["diag"]) or b["mix"] & (a["mix"] | a["diag"]):
        return False
    return not (a["window"] and b["window"] and a["even"] and b["even"])


def preamble(n_logical, outcome):
    """Measures an extra input qubit (id n_logical) first; its outcome is
    the signal of the X/Z chunks."""
    s = n_logical
    return {"cmds": [("M", s, 0.3, (), ())], "mix": set(), "diag": set(), "window": False, "even": False,
            "m": s}


def run_chunks(chunks, n_logical, outputs, outcome_of, inp, extra_input=False):
    cmds = [c for ch in chunks for c in ch["cmds"]]
    pat = W.Pattern(list(range(n_logical + (1 if extra_input else 0))), outputs, cmds)
    meas = [c[1] for c in cmds if c[0] == "M"]
    psi, probs = oc.run(pat, [outcome_of[q] for q in meas], inp)
    return psi, dict(zip(meas, probs))


def test_swaps_allowed_by_the_rule_keep_output_and_probabilities():
    shared = 0
    for seed in range(6):
        g = np.random.default_rng(7000 + seed)
        n = 5
        chunks, outputs = chunks_of(n, g, 40, even_share=0.3, signal_qubit=n)
        outcome_of = {ch["m"]: int(g.integers(2)) for ch in chunks if ch["window"]}
        outcome_of[n] = 1  # the X/Z chunks act
        pre = preamble(n, 1)
        # the extra qubit is an input in |+>-like superposition with the rest
        inp = W.gaussian_state(n + 1, g).astype(np.complex128)
        inp /= np.linalg.norm(inp)  # in FP64: the first M's p would carry the complex64 norm error
        psi0, p0 = run_chunks([pre] + chunks, n, outputs, outcome_of, inp, extra_input=True)
        order = list(chunks)
        swaps = 0
        for _ in range(400):
            i = int(g.integers(len(order) - 1))
            a, b = order[i], order[i + 1]
            if may_swap(a, b):
                shared += bool((a["mix"] | a["diag"]) & (b["mix"] | b["diag"]))
                order[i], order[i + 1] = b, a
                swaps += 1
        assert swaps > 50
        psi1, p1 = run_chunks([pre] + order, n, outputs, outcome_of, inp, extra_input=True)
        assert np.max(np.abs(psi1 - psi0)) <= 1e-12, seed
        for q in p0:
            assert abs(p1[q] - p0[q]) <= 1e-12, (seed, q)
    # swaps of steps that share a wire (only as signs) were exercised
    assert shared > 20, shared


def test_the_rule_forbids_what_does_not_commute():
    """A window and a CZ reading its wire, or an X and a Z on one wire, do
    not commute: swapping them changes the output."""
    g = np.random.default_rng(7200)
    n = 3
    inp = W.gaussian_state(n + 1, g).astype(np.complex128)
    inp /= np.linalg.norm(inp)
    pre = preamble(n, 1)
    win = {"cmds": [("N", 10), ("E", 0, 10), ("M", 0, 0.7, (), ()), ("X", 10, (0,))], "mix": {0}, "diag": set(),
           "window": True, "even": False, "m": 0}
    cz = {"cmds": [("E", 10, 1)], "mix": set(), "diag": {0, 1}, "window": False, "even": False, "m": None}
    cz_before = {"cmds": [("E", 0, 1)], "mix": set(), "diag": {0, 1}, "window": False, "even": False, "m": None}
    assert not may_swap(win, cz) and not may_swap(cz_before, win)
    oc_of = {0: 0, n: 1}
    a, _ = run_chunks([pre, win, cz], n, [10, 1, 2], oc_of, inp, extra_input=True)
    b, _ = run_chunks([pre, cz_before, win], n, [10, 1, 2], oc_of, inp, extra_input=True)
    assert np.max(np.abs(a - b)) > 1e-3
    x = {"cmds": [("X", 1, (n,))], "mix": {1}, "diag": set(), "window": False, "even": False, "m": None}
    z = {"cmds": [("Z", 1, (n,))], "mix": set(), "diag": {1}, "window": False, "even": False, "m": None}
    assert not may_swap(x, z)
    a, _ = run_chunks([pre, x, z], n, [0, 1, 2], {n: 1}, inp, extra_input=True)
    b, _ = run_chunks([pre, z, x], n, [0, 1, 2], {n: 1}, inp, extra_input=True)
    assert np.max(np.abs(a + b)) <= 1e-12  # XZ = -ZX


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
        pre = [{"cmds": [("E", 0, 1)], "mix": set(), "diag": {0, 1}, "window": False, "even": False, "m": None},
               {"cmds": [("E", 1, 2)], "mix": set(), "diag": {1, 2}, "window": False, "even": False, "m": None}]
        a = {"cmds": [("N", 3), ("E", 0, 3), ("E", 0, 3), ("M", 0, float(g.uniform(0, 6.28)), (), ()),
                      ("X", 3, (0,))], "mix": {0}, "diag": set(), "window": True, "even": True, "m": 0}
        b = {"cmds": [("N", 4), ("E", 2, 4), ("E", 2, 4), ("M", 2, float(g.uniform(0, 6.28)), (), ()),
                      ("X", 4, (2,))], "mix": {2}, "diag": set(), "window": True, "even": True, "m": 2}
        assert not may_swap(a, b)
        outcome_of = {0: int(g.integers(2)), 2: int(g.integers(2))}
        psi_ab, p_ab = run_chunks(pre + [a, b], n, [3, 1, 4], outcome_of, inp)
        psi_ba, p_ba = run_chunks(pre + [b, a], n, [3, 1, 4], outcome_of, inp)
        assert np.max(np.abs(psi_ab - psi_ba)) <= 1e-12
        worst = max(worst, abs(p_ab[0] - p_ba[0]), abs(p_ab[2] - p_ba[2]))
    assert worst > 1e-3
