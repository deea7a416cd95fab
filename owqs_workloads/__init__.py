"""Seeded synthetic workloads for one-way quantum computer (1WQC) pattern simulation.

This module only *builds inputs*: measurement patterns, measurement angles,
forced outcome strings and input state vectors.  It performs none of the
simulation arithmetic, so both the FP64 oracle (under ``oracle/``) and the HIP
library (``paper_1604_05659_amd``) can consume the same inputs without sharing
any simulation code.

Pattern model (Sec. 2.2 of the paper): a pattern is P = (V, I, O, A).  The
command list A is stored in *execution order* (first command first); the paper
writes patterns right to left.  Commands are tuples:

* ``('N', q)``                 prepare qubit q in |+>
* ``('E', u, v)``              controlled-Z between u and v
* ``('M', q, alpha, S, T)``    XY-plane measurement of q at angle alpha with
                               signal domains S (the ``s`` of Eq. 2) and T
                               (the ``t`` of Eq. 2); S, T are tuples of
                               previously measured qubit ids
* ``('X', q, S)``, ``('Z', q, S)`` Pauli corrections applied when the XOR of
                               the outcomes of the qubits in S is 1

Outcome strings are given per measurement command, in execution order.
Input states use qubit ``inputs[k]`` as bit k of the amplitude index; read-out
states use ``outputs[k]`` as bit k.

Seeds: every random draw comes from
``numpy.random.default_rng([160405659, config_id, purpose, index])`` with
purpose 0 = structure, 1 = angles, 2 = outcomes, 3 = input state.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_ROOT = 160405659
P_STRUCT, P_ANGLE, P_OUTCOME, P_INPUT = 0, 1, 2, 3

OP_N, OP_E, OP_M, OP_X, OP_Z = 0, 1, 2, 3, 4
OP_CODES = {"N": OP_N, "E": OP_E, "M": OP_M, "X": OP_X, "Z": OP_Z}


def rng(config_id: int, purpose: int, index: int = 0) -> np.random.Generator:
    """The seeded stream for (config, purpose, index)."""
    return np.random.default_rng([SEED_ROOT, int(config_id), int(purpose), int(index)])


@dataclass
class Pattern:
    """A 1WQC measurement pattern in execution order (see module docstring)."""

    inputs: List[int]
    outputs: List[int]
    cmds: List[tuple]
    name: str = ""

    # ---- structural queries (no simulation) ----
    def measured(self) -> List[int]:
        return [c[1] for c in self.cmds if c[0] == "M"]

    def n_meas(self) -> int:
        return sum(1 for c in self.cmds if c[0] == "M")

    def angles(self) -> np.ndarray:
        return np.array([c[2] for c in self.cmds if c[0] == "M"], dtype=np.float64)

    def with_angles(self, alphas: Sequence[float]) -> "Pattern":
        """Copy of the pattern with the M angles replaced (execution order)."""
        alphas = list(alphas)
        if len(alphas) != self.n_meas():
            raise ValueError("need one angle per M command")
        out, k = [], 0
        for c in self.cmds:
            if c[0] == "M":
                out.append(("M", c[1], float(alphas[k]), c[3], c[4]))
                k += 1
            else:
                out.append(c)
        return Pattern(list(self.inputs), list(self.outputs), out, self.name)

    def qubits(self) -> List[int]:
        seen, order = set(), []
        for q in self.inputs:
            if q not in seen:
                seen.add(q)
                order.append(q)
        for c in self.cmds:
            qs = (c[1], c[2]) if c[0] == "E" else (c[1],)
            for q in qs:
                if q not in seen:
                    seen.add(q)
                    order.append(q)
        return order

    def live_width_profile(self) -> List[int]:
        """Live width after each command under prepare-on-N / drop-on-M."""
        n = len(self.inputs)
        prof = []
        for c in self.cmds:
            if c[0] == "N":
                n += 1
            elif c[0] == "M":
                n -= 1
            prof.append(n)
        return prof

    def max_live(self) -> int:
        """Largest number of simultaneously live qubits (before each M)."""
        n = len(self.inputs)
        m = n
        for c in self.cmds:
            if c[0] == "N":
                n += 1
                m = max(m, n)
            elif c[0] == "M":
                n -= 1
        return m

    def counts(self) -> dict:
        d = {"N": 0, "E": 0, "M": 0, "X": 0, "Z": 0}
        for c in self.cmds:
            d[c[0]] += 1
        return d

    def nontrivial_count(self, outcomes: Sequence[int]) -> int:
        """N, E, M always count; X/Z only when their signal is 1."""
        res = {}
        mi = 0
        cnt = 0
        for c in self.cmds:
            if c[0] == "M":
                res[c[1]] = int(outcomes[mi]) & 1
                mi += 1
                cnt += 1
            elif c[0] in ("X", "Z"):
                s = 0
                for j in c[2]:
                    s ^= res[j]
                cnt += s
            else:
                cnt += 1
        return cnt

    # ---- text format v1 ----
    def to_text(self) -> str:
        lines = ["# owqs pattern v1" + (f" {self.name}" if self.name else "")]
        lines.append("inputs" + "".join(f" {q}" for q in self.inputs))
        lines.append("outputs" + "".join(f" {q}" for q in self.outputs))
        for c in self.cmds:
            if c[0] == "N":
                lines.append(f"N {c[1]}")
            elif c[0] == "E":
                lines.append(f"E {c[1]} {c[2]}")
            elif c[0] == "M":
                s = f"M {c[1]} {float(c[2])!r}"
                if c[3]:
                    s += " s:" + "".join(f" {j}" for j in c[3])
                if c[4]:
                    s += " t:" + "".join(f" {j}" for j in c[4])
                lines.append(s)
            else:
                s = f"{c[0]} {c[1]}"
                if c[2]:
                    s += " s:" + "".join(f" {j}" for j in c[2])
                lines.append(s)
        return "\n".join(lines) + "\n"

    @staticmethod
    def from_text(text: str) -> "Pattern":
        inputs: List[int] = []
        outputs: List[int] = []
        cmds: List[tuple] = []
        for raw in text.splitlines():
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            head = tok[0]
            if head == "inputs":
                inputs = [int(t) for t in tok[1:]]
                continue
            if head == "outputs":
                outputs = [int(t) for t in tok[1:]]
                continue
            if head == "N":
                cmds.append(("N", int(tok[1])))
            elif head == "E":
                cmds.append(("E", int(tok[1]), int(tok[2])))
            elif head in ("M", "X", "Z"):
                q = int(tok[1])
                rest = tok[2:]
                alpha = 0.0
                if head == "M":
                    alpha = float(rest[0])
                    rest = rest[1:]
                doms = {"s:": [], "t:": []}
                cur = None
                for t in rest:
                    if t in doms:
                        cur = t
                    else:
                        if cur is None:
                            raise ValueError(f"bad line: {raw}")
                        doms[cur].append(int(t))
                if head == "M":
                    cmds.append(("M", q, alpha, tuple(doms["s:"]), tuple(doms["t:"])))
                else:
                    if doms["t:"]:
                        raise ValueError(f"t-domain on a correction: {raw}")
                    cmds.append((head, q, tuple(doms["s:"])))
            else:
                raise ValueError(f"unknown command: {raw}")
        return Pattern(inputs, outputs, cmds)


@dataclass
class Workload:
    """A pattern plus the forced outcomes and the input state for one run."""

    pattern: Pattern
    outcomes: np.ndarray                 # uint8, one per M, execution order
    input_state: Optional[np.ndarray]    # complex64, 2^|I| amplitudes, or None when |I| = 0
    meta: dict = field(default_factory=dict)


# ---------------------------------------------------------------------------
# circuits of J(alpha) and CZ gates and their translation into patterns
# ---------------------------------------------------------------------------

def random_jcz_circuit(n_logical: int, n_j: int, n_cz: int, g: np.random.Generator,
                       angle_g: Optional[np.random.Generator] = None) -> List[tuple]:
    """n_j J(alpha) gates on uniform targets and n_cz CZ gates on uniform pairs,
    in a seeded random interleaving.  Angles are uniform in [0, 2pi)."""
    angle_g = angle_g if angle_g is not None else g
    gates: List[tuple] = []
    for _ in range(n_j):
        gates.append(("J", int(g.integers(n_logical)), 0.0))
    for _ in range(n_cz):
        a, b = g.choice(n_logical, size=2, replace=False)
        gates.append(("CZ", int(a), int(b)))
    perm = g.permutation(len(gates))
    gates = [gates[i] for i in perm]
    out = []
    for gt in gates:
        if gt[0] == "J":
            out.append(("J", gt[1], float(angle_g.uniform(0.0, 2.0 * math.pi))))
        else:
            out.append(gt)
    return out


def inverse_jcz_gates(gates: Sequence[tuple]) -> List[tuple]:
    """Gates of the inverse circuit, again using only J and CZ:
    CZ^-1 = CZ and J(a)^-1 = diag(1, e^{-ia}) H = J(0) J(-a) J(0), listed in
    application order (J(0) first)."""
    out: List[tuple] = []
    for g in reversed(list(gates)):
        if g[0] == "J":
            out.extend([("J", g[1], 0.0), ("J", g[1], -g[2]), ("J", g[1], 0.0)])
        else:
            out.append(g)
    return out


def circuit_to_pattern(n_logical: int, gates: Sequence[tuple], prepare_zero: bool = False,
                       name: str = "") -> Pattern:
    """Translate a J/CZ circuit into a pattern in execution order.

    J(alpha) on logical qubit q currently held by pattern qubit u becomes
    ``N w; E u w; M u (-alpha); X w s:u`` and w then holds q; CZ(a, b) becomes
    ``E`` on the current holders.  The N of each new qubit sits right before
    its first E, so the live width alternates between n and n+1.

    ``prepare_zero``: the logical qubits are not inputs; each starts as N then
    J(0), which turns |+> into |0>, so the circuit starts from |0...0>.
    """
    cmds: List[tuple] = []
    cur = list(range(n_logical))
    nxt = n_logical
    inputs = [] if prepare_zero else list(range(n_logical))

    def apply_j(q: int, alpha: float) -> None:
        nonlocal nxt
        u = cur[q]
        w = nxt
        nxt += 1
        cmds.append(("N", w))
        cmds.append(("E", u, w))
        cmds.append(("M", u, float(-alpha), (), ()))
        cmds.append(("X", w, (u,)))
        cur[q] = w

    if prepare_zero:
        for q in range(n_logical):
            cmds.append(("N", q))
        for q in range(n_logical):
            apply_j(q, 0.0)
    for gt in gates:
        if gt[0] == "J":
            apply_j(gt[1], gt[2])
        elif gt[0] == "CZ":
            cmds.append(("E", cur[gt[1]], cur[gt[2]]))
        else:
            raise ValueError(gt)
    return Pattern(inputs, list(cur), cmds, name)


def gaussian_state(n_qubits: int, g: np.random.Generator) -> np.ndarray:
    """Normalised complex Gaussian state, built in float64 then cast to complex64."""
    dim = 1 << n_qubits
    re = g.standard_normal(dim)
    im = g.standard_normal(dim)
    v = re + 1j * im
    v /= np.sqrt(np.sum(np.abs(v) ** 2))
    return v.astype(np.complex64)


def outcome_bits(n: int, g: np.random.Generator) -> np.ndarray:
    return g.integers(0, 2, size=n).astype(np.uint8)


# ---------------------------------------------------------------------------
# cluster-state patterns (Sec. 4.6: measured column by column)
# ---------------------------------------------------------------------------

def cluster_pattern(rows: int, cols: int, ks: np.ndarray, name: str = "") -> Pattern:
    """rows x cols rectangular cluster, all qubits prepared in |+> (no inputs),
    CZ on every nearest-neighbour edge, columns 0..cols-2 measured top to
    bottom at alpha = k*pi/4, column cols-1 the outputs.

    Signals follow the flow f(r, c) = (r, c+1): the s-domain of (r, c) is
    {(r, c-1)} and its t-domain is {(r-1, c-1), (r+1, c-1), (r, c-2)}
    restricted to measured qubits.  The outputs receive X^{s} Z^{t} with the
    same domains.  E commands are placed lazily: before (r, c) is measured its
    edges to (r, c+1) and (r+1, c) are applied, preparing qubits on first use.
    """
    qid = lambda r, c: c * rows + r  # noqa: E731
    prepared = set()
    cmds: List[tuple] = []

    def prep(q):
        if q not in prepared:
            prepared.add(q)
            cmds.append(("N", q))

    def domains(r, c):
        s = tuple([qid(r, c - 1)] if c - 1 >= 0 else [])
        t = []
        for (rr, cc) in ((r - 1, c - 1), (r + 1, c - 1), (r, c - 2)):
            if 0 <= rr < rows and 0 <= cc < cols - 1 and cc >= 0:
                t.append(qid(rr, cc))
        return s, tuple(t)

    for c in range(cols - 1):
        for r in range(rows):
            v = qid(r, c)
            prep(v)
            # edge to the right
            prep(qid(r, c + 1))
            cmds.append(("E", v, qid(r, c + 1)))
            # edge downwards
            if r + 1 < rows:
                prep(qid(r + 1, c))
                cmds.append(("E", v, qid(r + 1, c)))
            s, t = domains(r, c)
            alpha = float(ks[r, c]) * math.pi / 4.0
            cmds.append(("M", v, alpha, s, t))
    c = cols - 1
    for r in range(rows):
        prep(qid(r, c))
    for r in range(rows - 1):
        cmds.append(("E", qid(r, c), qid(r + 1, c)))
    for r in range(rows):
        s, t = domains(r, c)
        if s:
            cmds.append(("X", qid(r, c), s))
        if t:
            cmds.append(("Z", qid(r, c), t))
    outputs = [qid(r, cols - 1) for r in range(rows)]
    return Pattern([], outputs, cmds, name)


# ---------------------------------------------------------------------------
# layered ansatz (brick CZ pattern) used for gradients
# ---------------------------------------------------------------------------

def ansatz_gates(n_logical: int, layers: int, alphas: np.ndarray) -> List[tuple]:
    """``layers`` rounds of J(alpha) on every qubit followed by a CZ brick
    (pairs (2j, 2j+1) on even layers, (2j+1, 2j+2) on odd layers)."""
    gates: List[tuple] = []
    for l in range(layers):
        for q in range(n_logical):
            gates.append(("J", q, float(alphas[l, q])))
        start = 0 if l % 2 == 0 else 1
        for a in range(start, n_logical - 1, 2):
            gates.append(("CZ", a, a + 1))
    return gates


def ansatz_pattern(n_logical: int, layers: int, alphas: np.ndarray, name: str = "") -> Pattern:
    """The ansatz on |+>^n (each logical qubit is an N with no input)."""
    gates = ansatz_gates(n_logical, layers, alphas)
    cmds: List[tuple] = [("N", q) for q in range(n_logical)]
    inner = circuit_to_pattern(n_logical, gates, prepare_zero=False)
    cmds.extend(inner.cmds)
    return Pattern([], inner.outputs, cmds, name)


# ---------------------------------------------------------------------------
# the five workload recipes (configurable sizes so that tests can shrink them)
# ---------------------------------------------------------------------------

def plain_small(index: int = 0, n_logical: int = 4, n_j: int = 20, n_cz: int = 6) -> Workload:
    """Random J/CZ circuit on |0000> (prepared inside the pattern with J(0)),
    24 measured + 4 output qubits at the default sizes."""
    cid = 1
    gates = random_jcz_circuit(n_logical, n_j, n_cz, rng(cid, P_STRUCT, index), rng(cid, P_ANGLE, index))
    pat = circuit_to_pattern(n_logical, gates, prepare_zero=True, name=f"plain_small[{index}]")
    out = outcome_bits(pat.n_meas(), rng(cid, P_OUTCOME, index))
    return Workload(pat, out, None, {"gates": gates, "n_logical": n_logical})


def plain_large(index: int = 0, n_logical: int = 24, n_j: int = 2000, n_cz: int = 300) -> Workload:
    """Random J/CZ circuit on a normalised complex Gaussian input over
    n_logical qubits; live width alternates n_logical <-> n_logical + 1."""
    cid = 2
    gates = random_jcz_circuit(n_logical, n_j, n_cz, rng(cid, P_STRUCT, index), rng(cid, P_ANGLE, index))
    pat = circuit_to_pattern(n_logical, gates, prepare_zero=False, name=f"plain_large[{index}]")
    out = outcome_bits(pat.n_meas(), rng(cid, P_OUTCOME, index))
    psi = gaussian_state(n_logical, rng(cid, P_INPUT, index))
    return Workload(pat, out, psi, {"gates": gates, "n_logical": n_logical})


def cluster(index: int = 0, rows: int = 20, cols: int = 200) -> Workload:
    """rows x cols 2D cluster measured column by column at k*pi/4."""
    cid = 3
    ks = rng(cid, P_ANGLE, index).integers(0, 8, size=(rows, cols))
    pat = cluster_pattern(rows, cols, ks, name=f"cluster{rows}x{cols}[{index}]")
    out = outcome_bits(pat.n_meas(), rng(cid, P_OUTCOME, index))
    return Workload(pat, out, None, {"ks": ks, "rows": rows, "cols": cols})


def batched_random(index: int, w_lo: int = 8, w_hi: int = 20, c_lo: int = 50, c_hi: int = 800) -> Workload:
    """One pattern of the batched workload: width w ~ U{w_lo..w_hi} (w-1
    logical qubits), command budget C ~ U{c_lo..c_hi}; gates drawn with
    P(CZ) = 0.13 until 4*#J + #CZ >= C; Gaussian input."""
    cid = 4
    g = rng(cid, P_STRUCT, index)
    w = int(g.integers(w_lo, w_hi + 1))
    n_logical = w - 1
    budget = int(g.integers(c_lo, c_hi + 1))
    ag = rng(cid, P_ANGLE, index)
    gates: List[tuple] = []
    nj = ncz = 0
    while 4 * nj + ncz < budget:
        if n_logical >= 2 and g.random() < 0.13:
            a, b = g.choice(n_logical, size=2, replace=False)
            gates.append(("CZ", int(a), int(b)))
            ncz += 1
        else:
            gates.append(("J", int(g.integers(n_logical)), float(ag.uniform(0.0, 2.0 * math.pi))))
            nj += 1
    pat = circuit_to_pattern(n_logical, gates, prepare_zero=False, name=f"batched[{index}]")
    out = outcome_bits(pat.n_meas(), rng(cid, P_OUTCOME, index))
    psi = gaussian_state(n_logical, rng(cid, P_INPUT, index))
    return Workload(pat, out, psi, {"gates": gates, "n_logical": n_logical, "width": w})


def recognition(index: int = 0, n_logical: int = 12, n_j: int = 300, n_cz: int = 60) -> Workload:
    """Deterministic J/CZ pattern whose inputs are the n_logical logical
    qubits; the unitary is recovered from all 2^n_logical basis inputs.
    ``input_state`` is None: callers feed basis states."""
    cid = 5
    gates = random_jcz_circuit(n_logical, n_j, n_cz, rng(cid, P_STRUCT, index), rng(cid, P_ANGLE, index))
    pat = circuit_to_pattern(n_logical, gates, prepare_zero=False, name=f"recognition[{index}]")
    out = outcome_bits(pat.n_meas(), rng(cid, P_OUTCOME, index))
    return Workload(pat, out, None, {"gates": gates, "n_logical": n_logical})


def ansatz(index: int = 0, n_logical: int = 16, layers: int = 25, batch: int = 64) -> Tuple[Workload, np.ndarray]:
    """Layered ansatz on |+>^n; returns the workload (first angle set) and a
    (batch, n_meas) array of M angles (one row per angle set)."""
    cid = 6
    ag = rng(cid, P_ANGLE, index)
    gate_alphas = ag.uniform(0.0, 2.0 * math.pi, size=(batch, layers, n_logical))
    pat = ansatz_pattern(n_logical, layers, gate_alphas[0], name=f"ansatz{n_logical}x{layers}[{index}]")
    sets = np.stack([ansatz_pattern(n_logical, layers, gate_alphas[b]).angles() for b in range(batch)])
    out = outcome_bits(pat.n_meas(), rng(cid, P_OUTCOME, index))
    return Workload(pat, out, None, {"n_logical": n_logical, "layers": layers}), sets


def random_pattern(g: np.random.Generator, max_qubits: int = 10) -> Pattern:
    """A random pattern obeying D0-D3: random inputs, lazily prepared qubits,
    E between live qubits, M with random domains over measured qubits, and
    X/Z corrections with random domains."""
    nin = int(g.integers(0, 3))
    ids = list(range(max_qubits))
    inputs = ids[:nin]
    live = list(inputs)
    fresh = ids[nin:]
    measured = []
    cmds = []
    n_out = int(g.integers(1, 3))
    steps = 0
    while steps < 60:
        steps += 1
        r = g.random()
        if (r < 0.25 or len(live) < 2) and fresh:
            q = fresh.pop(0)
            cmds.append(("N", q))
            live.append(q)
        elif r < 0.55 and len(live) >= 2:
            a, b = g.choice(len(live), size=2, replace=False)
            cmds.append(("E", live[a], live[b]))
        elif r < 0.8 and len(live) > n_out:
            q = live.pop(int(g.integers(len(live))))
            def dom():
                if not measured:
                    return ()
                k = int(g.integers(0, min(3, len(measured)) + 1))
                return tuple(int(x) for x in g.choice(measured, size=k, replace=False))
            cmds.append(("M", q, float(g.uniform(0, 2 * math.pi)), dom(), dom()))
            measured.append(q)
        elif live and measured:
            q = live[int(g.integers(len(live)))]
            k = int(g.integers(1, min(2, len(measured)) + 1))
            d = tuple(int(x) for x in g.choice(measured, size=k, replace=False))
            cmds.append(("X" if g.random() < 0.5 else "Z", q, d))
        if not fresh and len(live) <= n_out:
            break
    while len(live) > n_out:
        q = live.pop(0)
        cmds.append(("M", q, float(g.uniform(0, 2 * math.pi)), (), ()))
        measured.append(q)
    return Pattern(inputs, list(live), cmds)


def basis_state(n_qubits: int, k: int) -> np.ndarray:
    v = np.zeros(1 << n_qubits, dtype=np.complex64)
    v[k] = 1.0
    return v


# ---------------------------------------------------------------------------
# Standard-form patterns (input to the reordering of Sec. 4.3)
# ---------------------------------------------------------------------------
def standard_form(pattern: Pattern) -> Pattern:
    """The same pattern with every N first, then every E, then the M commands
    in their order, then the corrections.  Valid when the corrections all come
    after the last M (each E involves qubits prepared before it and measured
    after it, so E and N commute to the front, Eqs. 15-16)."""
    cmds = pattern.cmds
    last_m = max((i for i, c in enumerate(cmds) if c[0] == "M"), default=-1)
    if any(c[0] in ("X", "Z") and i < last_m for i, c in enumerate(cmds)):
        raise ValueError("corrections before a measurement: not standardisable by commuting")
    ns = [c for c in cmds if c[0] == "N"]
    es = [c for c in cmds if c[0] == "E"]
    ms = [c for c in cmds if c[0] == "M"]
    cs = [c for c in cmds if c[0] in ("X", "Z")]
    return Pattern(list(pattern.inputs), list(pattern.outputs), ns + es + ms + cs, pattern.name + "/standard")


def random_standard_pattern(g: np.random.Generator, n_qubits: int = 9, n_in: int = 2, n_out: int = 2,
                            extra_edges: int = 4, max_dom: int = 2) -> Pattern:
    """A random pattern in standard form: a connected random graph on
    n_qubits (a random spanning tree plus extra edges), inputs the first
    n_in qubits, outputs the last n_out, measurements in a random order with
    s- and t-domains drawn from the qubits measured before, and X/Z
    corrections on the outputs with domains over measured qubits."""
    qs = list(range(n_qubits))
    perm = list(g.permutation(n_qubits))
    edges = set()
    for i in range(1, n_qubits):
        a, b = perm[i], perm[int(g.integers(i))]
        edges.add((min(a, b), max(a, b)))
    while len(edges) < n_qubits - 1 + extra_edges and len(edges) < n_qubits * (n_qubits - 1) // 2:
        a, b = (int(x) for x in g.choice(n_qubits, size=2, replace=False))
        edges.add((min(a, b), max(a, b)))
    inputs, outputs = qs[:n_in], qs[n_qubits - n_out:]
    meas = [q for q in g.permutation(n_qubits).tolist() if q not in outputs]
    cmds = [("N", q) for q in qs if q not in inputs]
    cmds += [("E", a, b) for a, b in sorted(edges)]
    done: List[int] = []
    for q in meas:
        ks = int(g.integers(0, min(max_dom, len(done)) + 1))
        kt = int(g.integers(0, min(max_dom, len(done)) + 1))
        s = tuple(int(x) for x in g.choice(done, size=ks, replace=False)) if ks else ()
        t = tuple(int(x) for x in g.choice(done, size=kt, replace=False)) if kt else ()
        cmds.append(("M", q, float(g.uniform(0, 2 * math.pi)), s, t))
        done.append(q)
    for q in outputs:
        for op in ("X", "Z"):
            k = int(g.integers(0, min(max_dom, len(done)) + 1))
            if k:
                cmds.append((op, q, tuple(int(x) for x in g.choice(done, size=k, replace=False))))
    return Pattern(inputs, outputs, cmds, "random_standard")


def disjoint_union(patterns: Sequence[Pattern], offset: int = 1000, name: str = "") -> Pattern:
    """Several patterns side by side on disjoint qubits (pattern k's ids plus
    k * offset), interleaved chunk by chunk (a chunk ends after an M and the
    corrections right after it, e.g. one J gate); inputs and outputs
    concatenated in pattern order.  The entanglement graph has at least one
    component per pattern, so the state stays a product across them."""
    shifted = []
    ins: List[int] = []
    outs: List[int] = []
    for k, pat in enumerate(patterns):
        d = k * offset
        cm = []
        for c in pat.cmds:
            if c[0] == "N":
                cm.append(("N", c[1] + d))
            elif c[0] == "E":
                cm.append(("E", c[1] + d, c[2] + d))
            elif c[0] == "M":
                cm.append(("M", c[1] + d, c[2], tuple(q + d for q in c[3]), tuple(q + d for q in c[4])))
            else:
                cm.append((c[0], c[1] + d, tuple(q + d for q in c[2])))
        shifted.append(cm)
        ins += [q + d for q in pat.inputs]
        outs += [q + d for q in pat.outputs]
    chunked = []
    for cm in shifted:
        chunks, cur = [], []
        for k, c in enumerate(cm):
            cur.append(c)
            nxt = cm[k + 1] if k + 1 < len(cm) else None
            if c[0] in ("M", "X", "Z") and not (nxt and nxt[0] in ("X", "Z")):
                if any(x[0] == "M" for x in cur):
                    chunks.append(cur)
                    cur = []
        if cur:
            chunks.append(cur)
        chunked.append(chunks)
    cmds = []
    for i in range(max((len(c) for c in chunked), default=0)):
        for chunks in chunked:
            if i < len(chunks):
                cmds.extend(chunks[i])
    return Pattern(ins, outs, cmds, name or "disjoint")
