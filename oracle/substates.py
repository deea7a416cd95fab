"""Sub-state execution (Sec. 4.1, Sec. 4.4.1, Fig. 8), written from the paper.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The system state is kept as a list of sub-states, each a vector over its own
qubits, the whole state being their tensor product (Sec. 4.1).  A new qubit
(N) is a sub-state of its own, |+>.  E on two qubits of different sub-states
first forms the tensor product of the two, then applies CZ (Sec. 4.4.1).  M
eliminates its qubit from its sub-state (Eqs. 11-12, the Fig. 6 compaction:
the remaining qubits keep their order); X and Z act inside the sub-state.
Sub-states are never split again (Sec. 5.1: the simulator does not
decompose).  A sub-state whose last qubit is measured leaves a scalar, kept
as a factor of the state.

Conventions: a sub-state is (qubits, vec) with bit k of the index of vec the
value of qubits[k].  The merge of u's sub-state A with v's sub-state B puts
B's qubits above A's: vec = kron(B.vec, A.vec).  Probabilities follow the
elimination oracle: p = sum |new|^2 with new = (psi0 + c psi1)/sqrt 2 over the
measured sub-state (each sub-state is normalised after every M, OWQS), or
p = 1/2 assumed with a sqrt 2 scale (EOWQS, Sec. 4.5).  Plain numpy: small
cases only.
"""
from __future__ import annotations

import cmath
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

MODE_OWQS = 0
MODE_EOWQS = 1
R2 = 1.0 / math.sqrt(2.0)


class SubStateError(RuntimeError):
    pass


class State:
    """The sub-state list of one run."""

    def __init__(self):
        self.subs: List[Tuple[List[int], np.ndarray]] = []
        self.scalar = 1.0 + 0j   # product of the sub-states whose qubits were all measured
        self.widest = 0          # largest sub-state width reached
        self.at_measure = []     # width of the measured qubit's sub-state, per M

    def find(self, q: int) -> int:
        for i, (qs, _) in enumerate(self.subs):
            if q in qs:
                return i
        raise SubStateError(f"qubit {q} is not live")

    def add(self, qubits: List[int], vec: np.ndarray):
        self.subs.append((list(qubits), np.asarray(vec, np.complex128).copy()))
        self.widest = max(self.widest, len(qubits))

    def merge(self, u: int, v: int) -> int:
        """Sub-state holding u and v (their tensor product if apart)."""
        a, b = self.find(u), self.find(v)
        if a == b:
            return a
        qa, va = self.subs[a]
        qb, vb = self.subs[b]
        merged = (qa + qb, np.kron(vb, va))
        for i in sorted((a, b), reverse=True):
            del self.subs[i]
        self.subs.append(merged)
        self.widest = max(self.widest, len(merged[0]))
        return len(self.subs) - 1

    def partition(self) -> List[List[int]]:
        return [list(qs) for qs, _ in self.subs]


def _bit_mask(n: int, b: int) -> np.ndarray:
    return ((np.arange(1 << n) >> b) & 1).astype(bool)


def _signal(dom, outcome_of) -> int:
    s = 0
    for q in dom:
        s ^= outcome_of[q]
    return s


def run(pattern, outcomes: Sequence[int], input_factors: Optional[Sequence[Tuple[Sequence[int], np.ndarray]]] = None,
        mode: int = MODE_OWQS, stop: Optional[int] = None):
    """Execute the pattern on sub-states.

    input_factors: the input state as a product of factors (qubits, vec),
    covering every input exactly once; None for a pattern without inputs.
    stop: number of commands to execute (None: all).
    Returns (State, probs), probs[m] the probability of the m-th M executed.
    """
    st = State()
    covered = []
    for qs, vec in (input_factors or []):
        if len(vec) != (1 << len(qs)):
            raise ValueError("input factor size mismatch")
        st.add(list(qs), vec)
        covered += list(qs)
    if sorted(covered) != sorted(pattern.inputs):
        raise ValueError("input factors must cover the inputs exactly once")
    outcome_of = {}
    probs = []
    m = 0
    cmds = pattern.cmds if stop is None else pattern.cmds[:stop]
    for c in cmds:
        op = c[0]
        if op == "N":
            st.add([c[1]], np.array([R2, R2]))
        elif op == "E":
            i = st.merge(c[1], c[2])
            qs, vec = st.subs[i]
            n = len(qs)
            both = _bit_mask(n, qs.index(c[1])) & _bit_mask(n, qs.index(c[2]))
            vec[both] = -vec[both]
        elif op in ("X", "Z"):
            if _signal(c[2], outcome_of):
                i = st.find(c[1])
                qs, vec = st.subs[i]
                n = len(qs)
                b = qs.index(c[1])
                if op == "X":
                    idx = np.arange(1 << n) ^ (1 << b)
                    st.subs[i] = (qs, vec[idx])
                else:
                    one = _bit_mask(n, b)
                    vec[one] = -vec[one]
        elif op == "M":
            v, alpha, sdom, tdom = c[1], c[2], c[3], c[4]
            s, t = _signal(sdom, outcome_of), _signal(tdom, outcome_of)
            theta = (-alpha if s else alpha) + (math.pi if t else 0.0)       # Eq. 2
            o = int(outcomes[m]) & 1
            coef = (-1.0 if o else 1.0) * cmath.exp(-1j * theta)           # Eqs. 11-12
            i = st.find(v)
            qs, vec = st.subs[i]
            n = len(qs)
            st.at_measure.append(n)
            b = qs.index(v)
            zero = ~_bit_mask(n, b)
            psi0 = vec[zero]                           # bit b removed, the rest in order
            psi1 = vec[np.nonzero(zero)[0] | (1 << b)]
            new = (psi0 + coef * psi1) * R2
            p = float(np.vdot(new, new).real)
            probs.append(p)
            if mode == MODE_OWQS:
                if p < 1e-12:
                    raise SubStateError(f"measurement {m} has zero probability")
                new = new / math.sqrt(p)
            else:
                new = new * math.sqrt(2.0)
            outcome_of[v] = o
            rest = qs[:b] + qs[b + 1:]
            del st.subs[i]
            if rest:
                st.subs.append((rest, new))
            else:
                st.scalar *= complex(new[0])
            m += 1
        else:
            raise ValueError(f"unknown command {op}")
    return st, np.array(probs)


def assemble(st: State, outputs: Sequence[int]) -> np.ndarray:
    """The full state over `outputs` (bit k = outputs[k]): the tensor product
    of the sub-states and the scalar."""
    n = len(outputs)
    pos = {q: k for k, q in enumerate(outputs)}
    out = np.full(1 << n, st.scalar, np.complex128)
    j = np.arange(1 << n)
    for qs, vec in st.subs:
        idx = np.zeros(1 << n, np.int64)
        for k, q in enumerate(qs):
            idx |= ((j >> pos[q]) & 1) << k
        out *= vec[idx]
    return out


def factor_in_order(qubits: Sequence[int], vec: np.ndarray, order: Sequence[int]) -> np.ndarray:
    """The same sub-state with its bits permuted to `order` (bit k = order[k])."""
    n = len(qubits)
    src = {q: k for k, q in enumerate(qubits)}
    j = np.arange(1 << n)
    idx = np.zeros(1 << n, np.int64)
    for k, q in enumerate(order):
        idx |= ((j >> k) & 1) << src[q]
    return np.asarray(vec)[idx]
