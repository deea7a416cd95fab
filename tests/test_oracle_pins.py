"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties the oracle to something other than itself: printed worked
examples (Fig. 8, Eq. 8, Eq. 21), closed forms (J(alpha), CNOT), invariants
(determinism of flow patterns, p = 1/2, norm, reordering), the Fig. 5 index
formula, the projectors of Eqs. 9-10, and an independent full-tensor brute
force.  No GPU.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc
from oracle import reference as ref

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SQ2 = math.sqrt(2.0)


def _den(s):
    return {"1": 1.0, "2": 2.0, "sqrt2": SQ2, "2sqrt2": 2 * SQ2}[s]


def _expected_from_substates(substates, slots):
    """Amplitude vector over the oracle's live slots (slot[k] = bit k) built as
    the product of the printed sub-states of the live qubits."""
    n = len(slots)
    bit_of = {q: k for k, q in enumerate(slots)}
    vec = np.zeros(1 << n, np.complex128)
    for i in range(1 << n):
        amp = 1.0 + 0j
        for sub in substates:
            qs = sub["qubits"]              # most significant first
            if not all(q in bit_of for q in qs):
                continue
            idx = 0
            for q in qs:
                idx = (idx << 1) | ((i >> bit_of[q]) & 1)
            amp *= sub["num"][idx] / _den(sub["den"])
        vec[i] = amp
    return vec


def fig8_pattern():
    """Eq. 23 in execution order, with lazy N (a qubit is prepared right
    before its first E)."""
    cmds = [("N", 3), ("E", 2, 3), ("M", 2, 0.0, (), ()),
            ("N", 4), ("E", 3, 4), ("E", 1, 3), ("M", 3, 0.0, (), ()),
            ("Z", 1, (2,)), ("Z", 4, (2,)), ("X", 4, (3,))]
    return W.Pattern([1, 2], [1, 4], cmds, "cnot_eq23")


def test_fig8_cnot_trace():
    gold = json.load(open(os.path.join(GOLD, "fig8_cnot.json")))
    pat = fig8_pattern()
    outcomes = [0, 1]
    psi_in = np.zeros(4, np.complex128)
    psi_in[3] = 1.0                           # |q2 q1> = |11>
    stages = {s["label"]: s["substates"] for s in gold["stages"]}
    # number of executed commands at each printed stage
    checkpoints = {"a": 0, "b": 2, "c": 3, "d": 6, "e": 7}
    for label, stop in checkpoints.items():
        live, slots, _ = oc.run(pat, outcomes, psi_in, stop=stop)
        exp = _expected_from_substates(stages[label], slots)
        np.testing.assert_allclose(live, exp, atol=1e-14, err_msg=f"stage {label}")
    # (a) also fixes N: preparing q3 gives q3 = (1, 1)/sqrt2
    live, slots, _ = oc.run(pat, outcomes, psi_in, stop=1)
    np.testing.assert_allclose(live, _expected_from_substates(stages["a"], slots), atol=1e-14)
    # (f) full run: outputs [q1, q4] with q1 at bit 0
    out, probs = oc.run(pat, outcomes, psi_in)
    np.testing.assert_allclose(out, _expected_from_substates(stages["f"], [1, 4]), atol=1e-14)
    np.testing.assert_allclose(probs, [0.5, 0.5], atol=1e-15)


def _signal_one_prefix(aux):
    """N aux; M aux at angle pi with outcome 1: probability 1, signal s_aux = 1."""
    return [("N", aux), ("M", aux, math.pi, (), ())]


def test_eq8_layout_and_bit_order():
    gold = json.load(open(os.path.join(GOLD, "eq8_layout.json")))
    arr = np.array([a + 1j * b for a, b in gold["array_num"]]) / _den(gold["array_den"])
    # the array is the ket expression with |b3 b2 b1> at index 4 b3 + 2 b2 + b1
    for ket, (re, im) in gold["kets"].items():
        assert abs(arr[int(ket, 2)] - (re + 1j * im) / _den(gold["array_den"])) < 1e-15
    assert abs(np.vdot(arr, arr) - 1) < 1e-15
    for target in (1, 2, 3):
        for op in ("X", "Z"):
            cmds = _signal_one_prefix(9) + [(op, target, (9,))]
            pat = W.Pattern([1, 2, 3], [1, 2, 3], cmds)
            out, probs = oc.run(pat, [1], arr)
            assert probs[0] == pytest.approx(1.0, abs=1e-15)
            # flip / phase the qubit q_target, i.e. ket position target-1 from the right
            exp = np.zeros(8, np.complex128)
            for ket, (re, im) in gold["kets"].items():
                bits = [int(ch) for ch in ket]                   # b3 b2 b1
                pos = 3 - target
                amp = (re + 1j * im) / _den(gold["array_den"])
                if op == "X":
                    bits[pos] ^= 1
                elif bits[pos] == 1:
                    amp = -amp
                exp[int("".join(map(str, bits)), 2)] += amp
            np.testing.assert_allclose(out, exp, atol=1e-14)


def test_eq21_compaction():
    g = np.random.default_rng(21)
    v = g.standard_normal(8) + 1j * g.standard_normal(8)
    v /= np.linalg.norm(v)
    a0, a1, b0, b1, a2, a3, b2, b3 = v                 # the Eq. 21 labelling
    for alpha in (0.0, 0.3, 2.5, -1.1):
        pat = W.Pattern([1, 2, 3], [1, 3], [("M", 2, alpha, (), ())])
        out, probs = oc.run(pat, [0], v)
        e = np.exp(-1j * alpha)
        raw = np.array([a0 + b0 * e, a1 + b1 * e, a2 + b2 * e, a3 + b3 * e]) / SQ2
        p0 = float(np.vdot(raw, raw).real)
        assert probs[0] == pytest.approx(p0, rel=1e-13)
        np.testing.assert_allclose(out, raw / math.sqrt(p0), atol=1e-14)


def test_measurement_probability_matches_projectors():
    """Eq. 13: p_o = <psi| P_o (x) I |psi> with P_0, P_1 as printed in Eqs. 9-10."""
    g = np.random.default_rng(13)
    for trial in range(20):
        v = g.standard_normal(4) + 1j * g.standard_normal(4)
        v /= np.linalg.norm(v)
        alpha = g.uniform(0, 2 * math.pi)
        for o in (0, 1):
            e = np.exp(-1j * alpha)
            p_mat = 0.5 * (np.array([[1, e], [np.conj(e), 1]]) if o == 0
                           else np.array([[1, -e], [-np.conj(e), 1]]))
            full = np.kron(np.eye(2), p_mat)            # measured qubit = bit 0
            p_exp = float(np.vdot(v, full @ v).real)
            pat = W.Pattern([1, 2], [2], [("M", 1, alpha, (), ())])
            _, probs = oc.run(pat, [o], v)
            assert probs[0] == pytest.approx(p_exp, rel=1e-12, abs=1e-15)


def test_window_with_odd_vw_count_has_probability_one_half():
    """N w; E's on v or w; M v with E(v, w) an odd number of times: the
    outcome has probability 1/2 for every input state and angle (the two
    halves of the new qubit are f (a + t) and +-f (a - t), Eqs. 11-13); with
    an even count it depends on the state.  Brute force: the projector of
    Eqs. 9-10 applied to the dense state after the CZs."""
    g = np.random.default_rng(1313)
    even_dev = 0.0
    for trial in range(40):
        k = int(g.integers(1, 4))                 # inputs 0 .. k-1, v = 0, w = k
        nvw = int(g.integers(1, 4))
        ev = [(0, k)] * nvw
        ev += [(0, x) for x in range(1, k) if g.integers(0, 2)]
        ev += [(k, y) for y in range(1, k) if g.integers(0, 2)]
        ev = [ev[i] for i in g.permutation(len(ev))]
        alpha = g.uniform(0, 2 * math.pi)
        psi = g.standard_normal(1 << k) + 1j * g.standard_normal(1 << k)
        psi /= np.linalg.norm(psi)
        dense = np.kron(np.array([1.0, 1.0]) / SQ2, psi)  # w is the top bit
        idx = np.arange(1 << (k + 1))
        for a, b in ev:
            dense = np.where(((idx >> a) & 1) & ((idx >> b) & 1), -dense, dense)
        for o in (0, 1):
            e = np.exp(-1j * alpha)
            p_mat = 0.5 * (np.array([[1, e], [np.conj(e), 1]]) if o == 0
                           else np.array([[1, -e], [-np.conj(e), 1]]))
            p_exp = float(np.vdot(dense, np.kron(np.eye(1 << k), p_mat) @ dense).real)
            cmds = [("N", k)] + [("E", a, b) for a, b in ev] + [("M", 0, alpha, (), ())]
            pat = W.Pattern(list(range(k)), list(range(1, k + 1)), cmds)
            _, probs = oc.run(pat, [o], psi)
            assert probs[0] == pytest.approx(p_exp, abs=1e-12)
            if nvw % 2:
                assert probs[0] == pytest.approx(0.5, abs=1e-12), (trial, ev)
            else:
                even_dev = max(even_dev, abs(probs[0] - 0.5))
    assert even_dev > 1e-3   # the even case is a real test of the state


def test_j_pattern_is_j_gate_for_both_outcomes():
    g = np.random.default_rng(2)
    for trial in range(10):
        alpha = g.uniform(0, 2 * math.pi)
        v = g.standard_normal(2) + 1j * g.standard_normal(2)
        v /= np.linalg.norm(v)
        pat = W.Pattern([1], [2], [("N", 2), ("E", 1, 2), ("M", 1, -alpha, (), ()), ("X", 2, (1,))])
        for o in (0, 1):
            out, probs = oc.run(pat, [o], v)
            exp = ref.H @ np.diag([1, np.exp(1j * alpha)]) @ v
            np.testing.assert_allclose(out, exp, atol=1e-14)
            assert probs[0] == pytest.approx(0.5, abs=1e-14)


def _cnot_expected(v):
    """CNOT with control q1 (bit 0) and target q2 (bit 1), the target then
    read as q4 at bit 1: |t c> -> |t xor c, c>."""
    out = np.zeros(4, np.complex128)
    for x in range(4):
        c, t = x & 1, (x >> 1) & 1
        out[c | ((t ^ c) << 1)] += v[x]
    return out


def test_cnot_pattern_all_outcomes_standard_and_reordered():
    g = np.random.default_rng(22)
    std = W.Pattern([1, 2], [1, 4],
                    [("N", 3), ("N", 4), ("E", 1, 3), ("E", 2, 3), ("E", 3, 4),
                     ("M", 2, 0.0, (), ()), ("M", 3, 0.0, (), ()),
                     ("Z", 1, (2,)), ("Z", 4, (2,)), ("X", 4, (3,))])     # Eq. 22
    lazy = fig8_pattern()                                                   # Eq. 23
    for trial in range(5):
        v = g.standard_normal(4) + 1j * g.standard_normal(4)
        v /= np.linalg.norm(v)
        for oc_bits in itertools.product((0, 1), repeat=2):
            a, pa = oc.run(std, oc_bits, v)
            b, pb = oc.run(lazy, oc_bits, v)
            exp = _cnot_expected(v)
            # Sec. 4.5: every branch gives the same unitary up to a global
            # phase.  Reading Eq. 22 right to left puts Z4 before X4, so the
            # branch s2 = s3 = 1 carries X Z = -Z X, i.e. a phase of -1.
            phase = -1.0 if oc_bits == (1, 1) else 1.0
            np.testing.assert_allclose(a, phase * exp, atol=1e-14)
            np.testing.assert_allclose(b, phase * exp, atol=1e-14)
            np.testing.assert_allclose(pa, [0.5, 0.5], atol=1e-14)
            np.testing.assert_allclose(pb, [0.5, 0.5], atol=1e-14)


def test_fig5_index_set():
    """The Fig. 5 index formula enumerates exactly the |11> quarter over the
    bits (u-1, v-1), and the oracle's E negates exactly that set."""
    g = np.random.default_rng(5)
    for n in range(2, 11):
        for u in range(2, n + 1):
            for v in range(1, u):
                lam = set()
                for i in range((1 << n) // 4):
                    j = i % (1 << (u - 2))
                    idx = ((j // (1 << (v - 1))) * (1 << v) + (1 << (v - 1)) + (j % (1 << (v - 1)))
                           + (i // (1 << (u - 2))) * (1 << u) + (1 << (u - 1)))
                    lam.add(idx)
                brute = {i for i in range(1 << n) if (i >> (u - 1)) & 1 and (i >> (v - 1)) & 1}
                assert lam == brute, (n, u, v)
                if n <= 6:
                    psi = g.standard_normal(1 << n) + 1j * g.standard_normal(1 << n)
                    pat = W.Pattern(list(range(1, n + 1)), list(range(1, n + 1)), [("E", u, v)])
                    # the E pattern keeps the norm, so feed a normalised vector
                    psi /= np.linalg.norm(psi)
                    out, _ = oc.run(pat, [], psi)
                    exp = psi.copy()
                    exp[sorted(lam)] *= -1
                    np.testing.assert_allclose(out, exp, atol=1e-15)


def test_oracle_matches_full_tensor_brute_force():
    g = np.random.default_rng(1604)
    checked = 0
    for trial in range(120):
        pat = W.random_pattern(g)
        nin = len(pat.inputs)
        v = None
        if nin:
            v = g.standard_normal(1 << nin) + 1j * g.standard_normal(1 << nin)
            v /= np.linalg.norm(v)
        outc = g.integers(0, 2, size=pat.n_meas())
        try:
            exp, pexp = ref.brute_force(pat, outc, v, return_probs=True)
        except (ZeroDivisionError, FloatingPointError):
            continue
        if np.min(pexp, initial=1.0) < 1e-6:
            continue
        got, pgot = oc.run(pat, outc, v)
        np.testing.assert_allclose(got, exp, atol=1e-11)
        np.testing.assert_allclose(pgot, pexp, atol=1e-11)
        checked += 1
    assert checked > 60


def test_plain_small_equals_circuit_for_sampled_outcomes():
    wl = W.plain_small()
    pat = wl.pattern
    exp = ref.circuit_state(4, wl.meta["gates"])
    g = np.random.default_rng(7)
    strings = [wl.outcomes, np.zeros(pat.n_meas(), np.uint8), np.ones(pat.n_meas(), np.uint8)]
    strings += [g.integers(0, 2, size=pat.n_meas()) for _ in range(10)]
    for s in strings:
        got, probs = oc.run(pat, s)
        np.testing.assert_allclose(got, exp, atol=1e-12)
        np.testing.assert_allclose(probs, 0.5, atol=1e-12)
        assert abs(np.vdot(got, got) - 1) < 1e-12


def test_plain_large_shape_equals_circuit_small_sizes():
    wl = W.plain_large(n_logical=6, n_j=60, n_cz=12)
    exp = ref.circuit_state(6, wl.meta["gates"], wl.input_state)
    inp = wl.input_state.astype(np.complex128)
    scale = np.linalg.norm(inp)
    for mode in (oc.MODE_OWQS, oc.MODE_EOWQS):
        got, probs = oc.run(wl.pattern, wl.outcomes, inp, mode=mode)
        # OWQS renormalises after each M; EOWQS keeps the input's norm
        want = exp / scale if mode == oc.MODE_OWQS else exp
        np.testing.assert_allclose(got, want, atol=1e-12)
        np.testing.assert_allclose(probs, 0.5, atol=1e-6)


def _cluster_circuit(ks, rows, cols):
    gates = []
    for r in range(rows - 1):
        gates.append(("CZ", r, r + 1))
    for c in range(cols - 1):
        for r in range(rows):
            gates.append(("J", r, -ks[r, c] * math.pi / 4))
        for r in range(rows - 1):
            gates.append(("CZ", r, r + 1))
    return gates


@pytest.mark.parametrize("rows,cols", [(3, 5), (4, 6), (1, 7)])
def test_cluster_determinism_and_circuit(rows, cols):
    wl = W.cluster(rows=rows, cols=cols)
    pat = wl.pattern
    exp = ref.circuit_state(rows, _cluster_circuit(wl.meta["ks"], rows, cols), start_plus=True)
    zero, pz = oc.run(pat, np.zeros(pat.n_meas(), np.uint8))
    np.testing.assert_allclose(zero, exp, atol=1e-12)          # all-zero branch: exact
    np.testing.assert_allclose(pz, 0.5, atol=1e-12)
    g = np.random.default_rng(rows * 100 + cols)
    for _ in range(12):
        s = g.integers(0, 2, size=pat.n_meas())
        got, probs = oc.run(pat, s)
        np.testing.assert_allclose(probs, 0.5, atol=1e-12)
        ph = np.vdot(exp, got)
        assert abs(abs(ph) - 1) < 1e-12                          # 1 - F = 0
        np.testing.assert_allclose(got, exp * ph, atol=1e-12)   # up to a global phase
    assert pat.max_live() == rows + 1                            # Sec. 4.6: m = N + 1


def test_reordering_invariance_standard_vs_lazy():
    """Proposition of Sec. 4.3: the standard form (all N, all E, then M, then
    corrections) and the lazy order give the same output."""
    for rows, cols in ((3, 4), (2, 6)):
        wl = W.cluster(rows=rows, cols=cols)
        pat = wl.pattern
        ns = [c for c in pat.cmds if c[0] == "N"]
        es = [c for c in pat.cmds if c[0] == "E"]
        rest = [c for c in pat.cmds if c[0] not in ("N", "E")]
        std = W.Pattern(pat.inputs, pat.outputs, ns + es + rest)
        g = np.random.default_rng(3)
        for _ in range(6):
            s = g.integers(0, 2, size=pat.n_meas())
            a, pa = oc.run(pat, s)
            b, pb = oc.run(std, s)
            np.testing.assert_allclose(a, b, atol=1e-12)
            np.testing.assert_allclose(pa, pb, atol=1e-12)
            np.testing.assert_allclose(a, ref.brute_force(std, s), atol=1e-11)


def test_eowqs_equals_owqs_on_flow_patterns():
    wl = W.plain_small(index=3)
    a, _ = oc.run(wl.pattern, wl.outcomes, mode=oc.MODE_OWQS)
    b, _ = oc.run(wl.pattern, wl.outcomes, mode=oc.MODE_EOWQS)
    np.testing.assert_allclose(a, b, atol=1e-12)


def test_parameter_shift_matches_finite_differences():
    wl, sets = W.ansatz(n_logical=4, layers=3, batch=1)
    alphas = sets[0]
    gs = oc.param_shift_grad(wl.pattern, wl.outcomes, alphas)
    gf = oc.central_fd_grad(wl.pattern, wl.outcomes, alphas, h=1e-4)
    np.testing.assert_allclose(gs, gf, atol=1e-7)
    # the loss does not depend on the outcome string of a flow pattern
    s = np.random.default_rng(0).integers(0, 2, size=wl.pattern.n_meas())
    assert oc.loss_at(wl.pattern, s, alphas) == pytest.approx(oc.loss_at(wl.pattern, wl.outcomes, alphas), abs=1e-12)
    # and matches the circuit
    gates = W.ansatz_gates(4, 3, -alphas.reshape(3, 4))
    psi = ref.circuit_state(4, gates, start_plus=True)
    assert oc.loss_z(psi) == pytest.approx(oc.loss_at(wl.pattern, wl.outcomes, alphas), abs=1e-12)


def test_pattern_rule_violations():
    v = np.array([1, 0], np.complex128)
    cases = [
        W.Pattern([1], [2], [("M", 2, 0.0, (), ())]),                                  # D2: M before N
        W.Pattern([1], [], [("M", 1, 0.0, (), ()), ("M", 1, 0.0, (), ())]),             # D1: measured twice
        W.Pattern([1], [2], [("N", 2), ("M", 1, 0.0, (), ()), ("E", 1, 2)]),            # D1: E on measured
        W.Pattern([1], [1], [("M", 1, 0.0, (), ())]),                                   # D3: measuring an output
        W.Pattern([1], [2], [("N", 2), ("M", 1, 0.0, (3,), ())]),                        # D0: unmeasured domain
        W.Pattern([1], [1, 2], [("N", 2)] + [("N", 2)]),                                # N twice
        W.Pattern([1], [1], [("N", 2)]),                                                # D3: unmeasured non-output
    ]
    for pat in cases:
        with pytest.raises(oc.OracleError) as e:
            oc.run(pat, [0, 0], v)
        assert e.value.code == -2
    # zero probability: |0> measured at angle 0 with the outcome that has p = 0
    plus = np.array([1, 1], np.complex128) / SQ2
    with pytest.raises(oc.OracleError) as e:
        oc.run(W.Pattern([1], [], [("M", 1, 0.0, (), ())]), [1], plus)
    assert e.value.code == -3
    # EOWQS on a non-deterministic measurement (|0> measured in the X-Y plane is fine: p = 1/2)
    out, p = oc.run(W.Pattern([1], [], [("M", 1, 0.7, (), ())]), [1], v, mode=oc.MODE_EOWQS)
    assert p[0] == pytest.approx(0.5)
    w = np.array([math.cos(0.3), math.sin(0.3)], np.complex128)
    with pytest.raises(oc.OracleError) as e:
        oc.run(W.Pattern([1], [], [("M", 1, 0.0, (), ())]), [0], w, mode=oc.MODE_EOWQS)
    assert e.value.code == -7


def test_seeded_outcome_stream_is_splitmix64():
    """The seeded outcome stream is SplitMix64 from its published definition;
    pinned to the reference implementation's outputs for state 1234567."""
    g = json.load(open(os.path.join(GOLD, "splitmix64_seed1234567.json")))
    want = [int(x) for x in g["outputs"]]
    assert oc.splitmix64(g["seed"], len(want)) == want
    bits = oc.outcomes_from_seed(g["seed"], len(want))
    assert bits.tolist() == [v >> 63 for v in want]
    # the bits of a long stream are balanced and differ between nearby seeds
    a, b = oc.outcomes_from_seed(7, 4096), oc.outcomes_from_seed(8, 4096)
    assert abs(a.mean() - 0.5) < 0.04 and abs(b.mean() - 0.5) < 0.04
    assert 0.4 < (a != b).mean() < 0.6


def test_sampled_outcomes_follow_the_bloch_sphere_probability():
    """Sampling (Fig. 6): outcome 0 exactly when u <= p_0.  For the qubit
    cos a |0> + e^{ib} sin a |1> measured in the XY plane at alpha, p_0 is
    (1 + sin 2a cos(b - alpha)) / 2 (Bloch vector (sin 2a cos b, sin 2a sin b,
    cos 2a) projected on (cos alpha, sin alpha, 0))."""
    g = np.random.default_rng(404)
    for a, b, alpha in [(0.3, 1.1, 0.4), (1.2, -0.7, 2.5), (0.785, 0.0, 0.0), (0.1, 2.0, 5.0)]:
        psi = np.array([math.cos(a), complex(math.cos(b), math.sin(b)) * math.sin(a)], np.complex128)
        p0 = 0.5 * (1.0 + math.sin(2 * a) * math.cos(b - alpha))
        pat = W.Pattern([0], [], [("M", 0, alpha, (), ())])
        for u in np.concatenate([np.linspace(0.0, 0.999, 37), [p0 - 1e-9, p0 + 1e-9]]):
            u = float(min(max(u, 0.0), 0.999999))
            _, probs, outc = oc.run_sampled(pat, [u], psi)
            assert outc[0] == (0 if u <= p0 else 1), (a, b, alpha, u, p0)
            assert probs[0] == pytest.approx(p0 if outc[0] == 0 else 1 - p0, abs=1e-12)
        # frequencies over many draws
        us = g.random(4000)
        zeros = sum(int(oc.run_sampled(pat, [float(u)], psi)[2][0] == 0) for u in us)
        sd = math.sqrt(4000 * p0 * (1 - p0)) + 1e-9
        assert abs(zeros - 4000 * p0) <= 5 * sd + 1


def test_sampled_runs_of_flow_patterns_are_deterministic():
    """Patterns with flow give the same output whatever is drawn (Sec. 4.5),
    and a drawn outcome string replayed as forced outcomes reproduces the run."""
    g = np.random.default_rng(405)
    wl = W.plain_small()
    want, _ = oc.run(wl.pattern, np.zeros(wl.pattern.n_meas(), np.uint8))
    for _ in range(5):
        u = g.random(wl.pattern.n_meas())
        got, probs, outc = oc.run_sampled(wl.pattern, u)
        np.testing.assert_allclose(got, want, atol=1e-12)
        np.testing.assert_allclose(probs, 0.5, atol=1e-12)
        replay, pr = oc.run(wl.pattern, outc)
        np.testing.assert_allclose(replay, got, atol=1e-12)
        np.testing.assert_allclose(pr, probs, atol=1e-12)
    # cluster patterns agree up to the global phase of signal-adapted angles
    cl = W.cluster(rows=4, cols=6)
    ref, _ = oc.run(cl.pattern, np.zeros(cl.pattern.n_meas(), np.uint8))
    got, _, outc = oc.run_sampled(cl.pattern, g.random(cl.pattern.n_meas()))
    assert abs(abs(np.vdot(ref, got)) - 1.0) < 1e-10
    assert outc.any() and not outc.all()
