"""ctypes wrapper of the complex128 C oracle (``owqs_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The C file follows Sec. 2.2 (commands, Eq. 2 signals, rules D0-D3),
Sec. 4.2 (qubit elimination with the operators of Eqs. 11-12, probability by
Eq. 13), Sec. 4.4 (implicit E, X, Z; Fig. 5 and the Fig. 6 compaction map) and
Sec. 4.5 (EOWQS: p = 1/2 assumed).  This module only marshals arrays and adds
the loss and gradient helpers used for the differentiated workload.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "owqs_oracle.c")
LIB = os.path.join(HERE, "libowqs_oracle.so")

MODE_OWQS = 0
MODE_EOWQS = 1
_OPS = {"N": 0, "E": 1, "M": 2, "X": 3, "Z": 4}

ERRORS = {
    -1: "invalid argument",
    -2: "pattern violates D0-D3",
    -3: "forced outcome has zero probability",
    -4: "width over the oracle limit",
    -5: "out of memory",
    -7: "EOWQS mode on a non-deterministic measurement",
}


class OracleError(RuntimeError):
    def __init__(self, code: int, cmd: int):
        super().__init__(f"oracle error {code} ({ERRORS.get(code, '?')}) at command {cmd}")
        self.code = code
        self.cmd = cmd


_M64 = (1 << 64) - 1


def splitmix64(seed: int, count: int) -> list:
    """The first `count` outputs of SplitMix64 (Steele, Lea and Flood, "Fast
    splittable pseudorandom number generators", OOPSLA 2014) started at
    `seed`: the state advances by the golden-ratio increment and each new
    state goes through the variant-13 64-bit finaliser."""
    out = []
    x = seed & _M64
    for _ in range(count):
        x = (x + 0x9E3779B97F4A7C15) & _M64
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        out.append(z ^ (z >> 31))
    return out


def outcomes_from_seed(seed: int, n_meas: int) -> np.ndarray:
    """Forced outcome bits of a seeded run: the top bit of each output."""
    return np.array([v >> 63 for v in splitmix64(seed, n_meas)], np.uint8)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP for the amplitude loops)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.owqs_oracle_run.restype = ctypes.c_int
        lib.owqs_oracle_run.argtypes = [
            ctypes.c_int, ip, ip, ip, dp, ip, ip, ip, ip, ip,
            ctypes.c_int, ip, ctypes.c_int, ip, dp, dp,
            ctypes.POINTER(ctypes.c_ubyte), dp, ctypes.c_int, ctypes.c_int,
            dp, dp, dp, ip, ip, ip]
        lib.owqs_oracle_set_threads.restype = ctypes.c_int
        lib.owqs_oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def set_threads(n: int) -> int:
    """Set the OpenMP thread count; returns the count in effect."""
    return _load().owqs_oracle_set_threads(int(n))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _arrays(pattern):
    n = len(pattern.cmds)
    op = np.zeros(n, np.int32)
    q0 = np.zeros(n, np.int32)
    q1 = np.zeros(n, np.int32)
    al = np.zeros(n, np.float64)
    so = np.zeros(n, np.int32)
    sl = np.zeros(n, np.int32)
    to = np.zeros(n, np.int32)
    tl = np.zeros(n, np.int32)
    dom = []
    for i, c in enumerate(pattern.cmds):
        op[i] = _OPS[c[0]]
        q0[i] = c[1]
        if c[0] == "E":
            q1[i] = c[2]
        elif c[0] == "M":
            al[i] = c[2]
            so[i], sl[i] = len(dom), len(c[3])
            dom.extend(c[3])
            to[i], tl[i] = len(dom), len(c[4])
            dom.extend(c[4])
        elif c[0] in ("X", "Z"):
            so[i], sl[i] = len(dom), len(c[2])
            dom.extend(c[2])
    dom_a = np.array(dom if dom else [0], np.int32)
    return op, q0, q1, al, so, sl, to, tl, dom_a


def run_sampled(pattern, uniforms: Sequence[float], input_state: Optional[np.ndarray] = None,
                stop: Optional[int] = None):
    """OWQS run whose outcomes are drawn (Fig. 6): the m-th M gives 0 when
    uniforms[m] <= p_0 (Eq. 13 of the outcome-0 branch, Eq. 11).  Returns
    (psi, probs, outcomes) on a full run, (live vector, slots, probs,
    outcomes) on a partial one; probs[m] is the probability of the drawn
    outcome."""
    u = np.ascontiguousarray(uniforms, np.float64)
    if u.size != pattern.n_meas():
        raise ValueError("one uniform per M command")
    res = run(pattern, np.zeros(pattern.n_meas(), np.uint8), input_state, MODE_OWQS, stop, _uniforms=u)
    return res


def run(pattern, outcomes: Sequence[int], input_state: Optional[np.ndarray] = None,
        mode: int = MODE_OWQS, stop: Optional[int] = None, _uniforms: Optional[np.ndarray] = None):
    """Execute the pattern.

    Full run (stop is None): returns (psi_out complex128 over the outputs in
    ``pattern.outputs`` bit order, probs float64 per M).
    Partial run (stop = number of commands to execute): returns
    (live vector, live slot list with slot[k] = qubit at bit k, probs).
    """
    lib = _load()
    op, q0, q1, al, so, sl, to, tl, dom = _arrays(pattern)
    nin = len(pattern.inputs)
    if input_state is None:
        if nin != 0:
            raise ValueError("pattern has inputs; an input state is required")
        input_state = np.ones(1, np.complex128)
    inp = np.asarray(input_state).astype(np.complex128)
    if inp.size != (1 << nin):
        raise ValueError("input size mismatch")
    in_re = np.ascontiguousarray(inp.real)
    in_im = np.ascontiguousarray(inp.imag)
    inputs = np.array(pattern.inputs if pattern.inputs else [0], np.int32)
    outputs = np.array(pattern.outputs if pattern.outputs else [0], np.int32)
    nmeas = pattern.n_meas()
    oc = np.zeros(max(nmeas, 1), np.uint8)
    oc[:nmeas] = np.asarray(outcomes, np.uint8)[:nmeas]
    probs = np.zeros(max(nmeas, 1), np.float64)
    if stop is None:
        cap = 1 << len(pattern.outputs)
    else:
        cap = 1 << pattern.max_live()
    out_re = np.zeros(cap, np.float64)
    out_im = np.zeros(cap, np.float64)
    slots = np.zeros(64, np.int32)
    n_live = np.zeros(1, np.int32)
    err = np.zeros(1, np.int32)
    rc = lib.owqs_oracle_run(
        len(pattern.cmds), _ptr(op, ctypes.c_int), _ptr(q0, ctypes.c_int), _ptr(q1, ctypes.c_int),
        _ptr(al, ctypes.c_double), _ptr(so, ctypes.c_int), _ptr(sl, ctypes.c_int),
        _ptr(to, ctypes.c_int), _ptr(tl, ctypes.c_int), _ptr(dom, ctypes.c_int),
        nin, _ptr(inputs, ctypes.c_int), len(pattern.outputs), _ptr(outputs, ctypes.c_int),
        _ptr(in_re, ctypes.c_double), _ptr(in_im, ctypes.c_double),
        _ptr(oc, ctypes.c_ubyte), None if _uniforms is None else _ptr(_uniforms, ctypes.c_double),
        int(mode), -1 if stop is None else int(stop),
        _ptr(out_re, ctypes.c_double), _ptr(out_im, ctypes.c_double), _ptr(probs, ctypes.c_double),
        _ptr(slots, ctypes.c_int), _ptr(n_live, ctypes.c_int), _ptr(err, ctypes.c_int))
    if rc != 0:
        raise OracleError(rc, int(err[0]))
    nm_done = nmeas if stop is None else sum(1 for c in pattern.cmds[:stop] if c[0] == "M")
    drawn = () if _uniforms is None else (oc[:nm_done].copy(),)
    if stop is None:
        return (out_re + 1j * out_im, probs[:nmeas].copy()) + drawn
    nl = int(n_live[0])
    return ((out_re[: 1 << nl] + 1j * out_im[: 1 << nl]), list(slots[:nl]), probs[:nm_done].copy()) + drawn


# ---------------------------------------------------------------------------
# observable and gradients for the differentiated workload
# ---------------------------------------------------------------------------

def z_weights(nout: int, obs: Optional[Sequence[int]] = None) -> np.ndarray:
    """W(x) = sum_{i in obs} (1 - 2 x_i): the diagonal of sum_i Z_i."""
    obs = list(range(nout)) if obs is None else list(obs)
    x = np.arange(1 << nout)
    w = np.zeros(1 << nout, np.float64)
    for i in obs:
        w += 1.0 - 2.0 * ((x >> i) & 1)
    return w


def loss_z(psi: np.ndarray, obs: Optional[Sequence[int]] = None) -> float:
    """sum_i <Z_i> over the output qubits (bit i of the read-out index)."""
    nout = int(round(math.log2(psi.size)))
    return float(np.sum(z_weights(nout, obs) * np.abs(psi) ** 2))


def loss_at(pattern, outcomes, alphas, input_state=None, mode=MODE_EOWQS, obs=None) -> float:
    psi, _ = run(pattern.with_angles(alphas), outcomes, input_state, mode)
    return loss_z(psi, obs)


def param_shift_grad(pattern, outcomes, alphas, input_state=None, mode=MODE_EOWQS,
                     obs=None, indices: Optional[Sequence[int]] = None) -> np.ndarray:
    """dL/d(alpha_k) for the M angles by the two-term shift rule.

    With p fixed (EOWQS), the output is affine in e^{-i theta_k} (Eqs. 11-12),
    so L = a + b cos(theta_k) + c sin(theta_k) and, since theta_k = +-alpha_k
    + const (Eq. 2), dL/dalpha = [L(alpha + pi/2) - L(alpha - pi/2)] / 2
    exactly.
    """
    alphas = np.asarray(alphas, np.float64)
    idx = range(alphas.size) if indices is None else indices
    g = np.zeros(alphas.size, np.float64)
    for k in idx:
        a = alphas.copy()
        a[k] += math.pi / 2
        lp = loss_at(pattern, outcomes, a, input_state, mode, obs)
        a[k] -= math.pi
        lm = loss_at(pattern, outcomes, a, input_state, mode, obs)
        g[k] = 0.5 * (lp - lm)
    return g


def central_fd_grad(pattern, outcomes, alphas, h=1e-4, input_state=None, mode=MODE_EOWQS,
                    obs=None, indices: Optional[Sequence[int]] = None) -> np.ndarray:
    alphas = np.asarray(alphas, np.float64)
    idx = range(alphas.size) if indices is None else indices
    g = np.zeros(alphas.size, np.float64)
    for k in idx:
        a = alphas.copy()
        a[k] += h
        lp = loss_at(pattern, outcomes, a, input_state, mode, obs)
        a[k] -= 2 * h
        lm = loss_at(pattern, outcomes, a, input_state, mode, obs)
        g[k] = (lp - lm) / (2 * h)
    return g
