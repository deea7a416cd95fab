"""Generalised flow (gflow) of a pattern's open graph, by brute force.

TEST INFRASTRUCTURE ONLY (see the package docstring).

EOWQS (Sec. 4.5) skips the probability of every measurement because, for
patterns with a gflow (Browne, Kashefi, Mhalla and Perdrix, "Generalized flow
and determinism in measurement-based quantum computation", 2007; reference
[13] of the paper), every branch has probability 1/2.  For measurements in
the XY plane a gflow of the open graph (G, I, O) is a map g from the measured
qubits to subsets of the non-input qubits and an order < such that, for every
measured i:
  (g1) every j in g(i) comes after i;
  (g2) every j != i with an odd number of neighbours in g(i) comes after i;
  (g3) i has an odd number of neighbours in g(i).
Here the order is the pattern's own measurement order (outputs come after
every measurement), which is what EOWQS needs: measuring i is then an
unbiased coin given every earlier outcome.

This module writes the definition out and searches it exhaustively: every
subset of the allowed qubits, every total order.  Small graphs only.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional, Sequence, Set


def open_graph(pattern):
    """(qubits, neighbours, inputs, outputs, measurement order) of a pattern;
    an edge is an odd number of E commands on a pair."""
    nbr: Dict[int, Set[int]] = {}
    qubits = set(pattern.inputs) | set(pattern.outputs)
    for c in pattern.cmds:
        qubits.add(c[1])
        if c[0] == "E":
            qubits.add(c[2])
            nbr.setdefault(c[1], set()).symmetric_difference_update({c[2]})
            nbr.setdefault(c[2], set()).symmetric_difference_update({c[1]})
    for q in qubits:
        nbr.setdefault(q, set())
    order = [c[1] for c in pattern.cmds if c[0] == "M"]
    return sorted(qubits), nbr, set(pattern.inputs), set(pattern.outputs), order


def odd(nbr, k: Sequence[int]) -> Set[int]:
    """Qubits with an odd number of neighbours in k."""
    out: Set[int] = set()
    for q in k:
        out ^= nbr[q]
    return out


def witness(nbr, inputs, i: int, before: Set[int], after: Set[int]) -> Optional[List[int]]:
    """A set K of non-input qubits, all in `after`, with odd(K) meeting
    before + {i} exactly in {i}; None if there is none (exhaustive)."""
    allowed = sorted(q for q in after if q not in inputs)
    if len(allowed) > 18:
        raise ValueError("too many candidate qubits for the exhaustive search")
    guard = before | {i}
    for r in range(len(allowed) + 1):
        for k in itertools.combinations(allowed, r):
            if odd(nbr, k) & guard == {i}:
                return list(k)
    return None


def certify_order(pattern) -> List[Optional[List[int]]]:
    """For each M in execution order: a witness g(i) for the pattern's own
    measurement order (later measurements and the outputs), or None."""
    qubits, nbr, ins, outs, order = open_graph(pattern)
    res = []
    for k, i in enumerate(order):
        before = set(order[:k])
        after = set(order[k + 1:]) | outs
        res.append(witness(nbr, ins, i, before, after))
    return res


def gflow_exists(pattern) -> bool:
    """Some total order of the measured qubits admits a witness for each
    (a gflow's partial order always extends to a total one).  Exhaustive over
    orders: small graphs only."""
    qubits, nbr, ins, outs, order = open_graph(pattern)
    meas = sorted(order)
    for perm in itertools.permutations(meas):
        ok = True
        for k, i in enumerate(perm):
            if witness(nbr, ins, i, set(perm[:k]), set(perm[k + 1:]) | outs) is None:
                ok = False
                break
        if ok:
            return True
    return False


def causal_flow_exists(pattern) -> bool:
    """As gflow_exists with every g(i) a single qubit (causal flow)."""
    qubits, nbr, ins, outs, order = open_graph(pattern)
    meas = sorted(order)
    for perm in itertools.permutations(meas):
        ok = True
        for k, i in enumerate(perm):
            before = set(perm[:k]) | {i}
            after = [q for q in set(perm[k + 1:]) | outs if q not in ins]
            if not any(odd(nbr, [j]) & before == {i} for j in after):
                ok = False
                break
        if ok:
            return True
    return False
