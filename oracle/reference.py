"""Independent numpy FP64 references (no elimination, no reordering).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``brute_force``   -- full-tensor execution over every qubit of the pattern.
  All non-input qubits start in |+> (Sec. 2.2, N), E is the CZ matrix of
  Sec. 2.1, X and Z the Pauli matrices, and each M applies the projector
  P_o = |w_o><w_o| of Eqs. 9-10 (w_0 = (1, e^{i theta})/sqrt 2,
  w_1 = (1, -e^{i theta})/sqrt 2, theta per Eq. 2) and renormalises (Eqs. 3-4).
  A measured qubit is then exactly |w_o>, so the final state of the outputs is
  read by contracting each measured qubit with <w_o|.
* ``circuit_state`` -- state-vector simulation of a J/CZ circuit, with
  J(alpha) = H diag(1, e^{i alpha}) and CZ = diag(1, 1, 1, -1) (Sec. 2.1).

Both are written from the definitions, in a form unrelated to the C oracle.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence

import numpy as np

H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def _apply_1q(psi: np.ndarray, bit: int, u: np.ndarray) -> np.ndarray:
    v = psi.reshape(-1, 2, 1 << bit)
    return np.einsum("ab,ibj->iaj", u, v).reshape(-1)


def _cz(psi: np.ndarray, b1: int, b2: int) -> np.ndarray:
    idx = np.arange(psi.size)
    sign = np.where(((idx >> b1) & 1) & ((idx >> b2) & 1), -1.0, 1.0)
    return psi * sign


def projector(theta: float, o: int) -> np.ndarray:
    """P_0 and P_1 of Eqs. 9-10 at angle theta."""
    e = np.exp(-1j * theta)
    if o == 0:
        return 0.5 * np.array([[1, e], [np.conj(e), 1]], dtype=np.complex128)
    return 0.5 * np.array([[1, -e], [-np.conj(e), 1]], dtype=np.complex128)


def basis_vector(theta: float, o: int) -> np.ndarray:
    """|w_o>: the eigenvector spanning the range of P_o (Eqs. 9-10)."""
    return np.array([1.0, (-1.0) ** o * np.exp(1j * theta)], dtype=np.complex128) / math.sqrt(2.0)


def brute_force(pattern, outcomes: Sequence[int], input_state: Optional[np.ndarray] = None,
                return_probs: bool = False):
    """Full-tensor reference; returns the normalised output state (outputs[k]
    at bit k) and optionally the per-M outcome probabilities."""
    qubits = pattern.qubits()
    if len(qubits) > 16:
        raise ValueError("brute force limited to 16 qubits")
    pos: Dict[int, int] = {q: k for k, q in enumerate(qubits)}
    nin = len(pattern.inputs)
    ntot = len(qubits)
    if nin:
        psi_in = np.asarray(input_state).astype(np.complex128)
    else:
        psi_in = np.ones(1, np.complex128)
    plus = np.ones(1 << (ntot - nin), np.complex128) / math.sqrt(2.0) ** (ntot - nin)
    # inputs occupy bits 0..nin-1 (qubits() lists inputs first)
    psi = np.kron(plus, psi_in)
    res: Dict[int, int] = {}
    thetas: Dict[int, float] = {}
    probs = []
    mi = 0
    for c in pattern.cmds:
        if c[0] == "N":
            continue                        # already |+> from the start
        if c[0] == "E":
            psi = _cz(psi, pos[c[1]], pos[c[2]])
        elif c[0] in ("X", "Z"):
            s = 0
            for j in c[2]:
                s ^= res[j]
            if s:
                psi = _apply_1q(psi, pos[c[1]], PX if c[0] == "X" else PZ)
        elif c[0] == "M":
            s = 0
            for j in c[3]:
                s ^= res[j]
            t = 0
            for j in c[4]:
                t ^= res[j]
            theta = (-1.0) ** s * c[2] + t * math.pi          # Eq. 2
            o = int(outcomes[mi]) & 1
            mi += 1
            proj = projector(theta, o)
            new = _apply_1q(psi, pos[c[1]], proj)
            p = float(np.vdot(new, new).real) / float(np.vdot(psi, psi).real)
            probs.append(p)
            psi = new / math.sqrt(float(np.vdot(new, new).real))
            res[c[1]] = o
            thetas[c[1]] = theta
    # contract every measured qubit with <w_o|, highest position first
    for q in sorted(res, key=lambda q: -pos[q]):
        w = basis_vector(thetas[q], res[q]).conj()
        b = pos[q]
        v = psi.reshape(-1, 2, 1 << b)
        psi = np.einsum("a,iaj->ij", w, v).reshape(-1)
        # positions above b shift down by one
        for qq in pos:
            if pos[qq] > b:
                pos[qq] -= 1
        pos[q] = -1
    # now only outputs remain; reorder to outputs[k] at bit k
    nout = len(pattern.outputs)
    live = sorted((p_, q) for q, p_ in pos.items() if p_ >= 0)
    assert len(live) == nout
    where = {q: p_ for p_, q in live}
    out = np.zeros(1 << nout, np.complex128)
    for x in range(1 << nout):
        src = 0
        for k, q in enumerate(pattern.outputs):
            if (x >> k) & 1:
                src |= 1 << where[q]
        out[x] = psi[src]
    out /= math.sqrt(float(np.vdot(out, out).real))
    if return_probs:
        return out, np.array(probs)
    return out


def j_matrix(alpha: float) -> np.ndarray:
    """J(alpha) = H diag(1, e^{i alpha})."""
    return H @ np.diag([1.0, np.exp(1j * alpha)])


def circuit_state(n_logical: int, gates: Sequence[tuple], input_state: Optional[np.ndarray] = None,
                  start_plus: bool = False) -> np.ndarray:
    """Run a J/CZ circuit; logical qubit k is bit k.  Starts from
    ``input_state``, or |0...0>, or |+...+> when ``start_plus``."""
    dim = 1 << n_logical
    if input_state is not None:
        psi = np.asarray(input_state).astype(np.complex128).copy()
    elif start_plus:
        psi = np.ones(dim, np.complex128) / math.sqrt(dim)
    else:
        psi = np.zeros(dim, np.complex128)
        psi[0] = 1.0
    for g in gates:
        if g[0] == "J":
            psi = _apply_1q(psi, g[1], j_matrix(g[2]))
        elif g[0] == "CZ":
            psi = _cz(psi, g[1], g[2])
        elif g[0] == "H":
            psi = _apply_1q(psi, g[1], H)
        else:
            raise ValueError(g)
    return psi


def circuit_unitary(n_logical: int, gates: Sequence[tuple]) -> np.ndarray:
    """Columns U[:, k] = circuit applied to |k> (dense; small n only)."""
    dim = 1 << n_logical
    u = np.zeros((dim, dim), np.complex128)
    for k in range(dim):
        e = np.zeros(dim, np.complex128)
        e[k] = 1.0
        u[:, k] = circuit_state(n_logical, gates, e)
    return u
