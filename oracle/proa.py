"""Pattern reordering (PROA, Sec. 4.3), written from the paper's description.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A pattern in standard form (all N, then all E, then the M commands, then the
corrections) is reordered so that each measured qubit is entangled with its
neighbours only just before it is measured (the Proposition of Sec. 4.3,
Eqs. 14-17).  Qubits start in singleton sub-states; choosing v merges the
sub-states of v and of its neighbours not yet entangled with it into the
measurement state-space MS(v), then v is measured and removed.  Among the
ready qubits (all measurement dependencies resolved) the one of least cost
(Eq. 18) is chosen:

  flag = 1:  alpha |MS(v)| + beta OS(v) - gamma SS(v)
  flag = 0:  alpha (|MS(v)| + 1) delta + beta OS(v) - gamma SS(v)

OS(v): edges from v to output qubits; SS(v): unmeasured qubits whose
measurement depends on v; flag = 1 when v already belongs to a sub-state made
by an earlier step.  Ties go to the smallest qubit id.  The weights default to
|O|, |O|, 0.5, |O| and alpha is swept |O|, |O|-1, ..., 1 (Sec. 5), keeping
the order with the smallest largest state-space (the first such alpha).
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple


def _graph(pattern):
    nbr: Dict[int, set] = {}
    qubits = set(pattern.inputs) | set(pattern.outputs)
    for c in pattern.cmds:
        qubits.add(c[1])
        if c[0] == "E":  # E twice is the identity: an edge is an odd number of E's
            qubits.add(c[2])
            nbr.setdefault(c[1], set()).symmetric_difference_update({c[2]})
            nbr.setdefault(c[2], set()).symmetric_difference_update({c[1]})
    for q in qubits:
        nbr.setdefault(q, set())
    return qubits, nbr


def _deps(pattern):
    """deps[v]: qubits whose outcomes the measurement of v depends on."""
    deps = {}
    for c in pattern.cmds:
        if c[0] == "M":
            deps[c[1]] = set(c[3]) | set(c[4])
    return deps


def order_once(pattern, alpha: float, beta: float, gamma: float, delta: float,
               ignore_dependencies: bool = False) -> Tuple[List[int], List[List[int]]]:
    """One PROA pass: the measurement order and each step's state-space."""
    qubits, nbr = _graph(pattern)
    outputs = set(pattern.outputs)
    deps = _deps(pattern)
    to_measure = [q for q in sorted(qubits) if q not in outputs]
    dependents = {v: {u for u in deps if v in deps[u]} for v in qubits}
    sub = {q: frozenset([q]) for q in qubits}          # qubit -> its sub-state
    pending = {q: set(nbr[q]) for q in qubits}          # neighbours not yet entangled
    touched = set()
    measured: set = set()
    order, spaces = [], []
    for _ in range(len(to_measure)):
        ready = [v for v in to_measure if v not in measured and
                 (ignore_dependencies or deps.get(v, set()) <= measured)]
        if not ready:
            raise ValueError("no measurable qubit: circular dependencies")
        best = None
        for v in ready:
            ms = set(sub[v])
            for u in pending[v]:
                ms |= sub[u]
            os_ = sum(1 for u in nbr[v] if u in outputs)
            ss = sum(1 for u in dependents[v] if u not in measured)
            if v in touched:
                cost = alpha * len(ms) + beta * os_ - gamma * ss
            else:
                cost = alpha * ((len(ms) + 1) * delta) + beta * os_ - gamma * ss
            if best is None or cost < best[0]:
                best = (cost, v, ms)
        _, v, ms = best
        order.append(v)
        spaces.append(sorted(ms))
        for u in list(pending[v]):
            pending[u].discard(v)
        pending[v].clear()
        rest = frozenset(ms - {v})
        for u in rest:
            sub[u] = rest
        touched |= ms
        measured.add(v)
    return order, spaces


def proa(pattern, weights: Optional[Sequence[float]] = None, ignore_dependencies: bool = False):
    """Returns (order, state-spaces, largest state-space size m, alpha used)."""
    n_out = len(pattern.outputs)
    if weights is not None:
        a, b, g, d = weights
        order, spaces = order_once(pattern, a, b, g, d, ignore_dependencies)
        return order, spaces, max((len(s) for s in spaces), default=0), a
    best = None
    base = max(n_out, 1)
    for k in range(base):
        a = float(base - k)
        order, spaces = order_once(pattern, a, float(base), 0.5, float(base), ignore_dependencies)
        m = max((len(s) for s in spaces), default=0)
        if best is None or m < best[2]:
            best = (order, spaces, m, a)
    return best


def sub_states_along(pattern, order: Sequence[int]):
    """Replay a given order: the state-space of each step and the sub-states
    (of unmeasured qubits) after it."""
    qubits, nbr = _graph(pattern)
    sub = {q: frozenset([q]) for q in qubits}
    pending = {q: set(nbr[q]) for q in qubits}
    measured = set()
    spaces, after = [], []
    for v in order:
        ms = set(sub[v])
        for u in pending[v]:
            ms |= sub[u]
        for u in list(pending[v]):
            pending[u].discard(v)
        pending[v].clear()
        rest = frozenset(ms - {v})
        for u in rest:
            sub[u] = rest
        measured.add(v)
        spaces.append(sorted(ms))
        live = {sub[q] for q in qubits if q not in measured}
        after.append(sorted(sorted(s) for s in live))
    return spaces, after


def reordered_pattern(pattern, order: Sequence[int], positive_branch: bool = False):
    """The executable pattern for a measurement order: before measuring v,
    prepare (N) the qubits of its state-space not prepared yet and apply its
    remaining E's; after the last M, prepare the remaining outputs, apply the
    remaining E's, then the corrections in their original order.  With
    positive_branch (every outcome 0, EOWQS, Sec. 4.5) the signal domains and
    corrections are dropped: every signal is 0."""
    import owqs_workloads as W
    qubits, nbr = _graph(pattern)
    m_cmd = {c[1]: c for c in pattern.cmds if c[0] == "M"}
    prepared = set(pattern.inputs)
    pending = {q: set(nbr[q]) for q in qubits}
    cmds = []

    def prep(q):
        if q not in prepared:
            cmds.append(("N", q))
            prepared.add(q)

    for v in order:
        prep(v)
        for u in sorted(pending[v]):
            prep(u)
            cmds.append(("E", v, u))
            pending[u].discard(v)
        pending[v].clear()
        c = m_cmd[v]
        cmds.append((c[0], c[1], c[2], (), ()) if positive_branch else c)
    for q in sorted(pattern.outputs):
        prep(q)
    for q in sorted(qubits):
        for u in sorted(pending[q]):
            if u > q:
                cmds.append(("E", q, u))
    for c in pattern.cmds:
        if c[0] in ("X", "Z") and not positive_branch:
            cmds.append(c)
    return W.Pattern(list(pattern.inputs), list(pattern.outputs), cmds)
