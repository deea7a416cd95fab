"""The seeded workload generators: sizes, structure and reproducibility."""
import numpy as np

import owqs_workloads as W
from oracle import reference as ref


def test_plain_small_structure():
    wl = W.plain_small()
    p = wl.pattern
    assert p.counts() == {"N": 28, "E": 30, "M": 24, "X": 24, "Z": 0}
    assert len(p.outputs) == 4 and p.n_meas() == 24 and p.max_live() <= 8


def test_plain_large_structure():
    wl = W.plain_large()
    p = wl.pattern
    assert p.counts() == {"N": 2000, "E": 2300, "M": 2000, "X": 2000, "Z": 0}
    assert len(p.inputs) == 24 and len(p.outputs) == 24 and p.max_live() == 25
    assert wl.input_state.dtype == np.complex64 and wl.input_state.size == 1 << 24
    assert abs(np.linalg.norm(wl.input_state.astype(np.complex128)) - 1) < 1e-6


def test_cluster_structure():
    wl = W.cluster()
    p = wl.pattern
    assert p.counts() == {"N": 4000, "E": 7780, "M": 3980, "X": 20, "Z": 20}
    assert p.max_live() == 21


def test_recognition_and_ansatz_structure():
    p = W.recognition().pattern
    assert p.counts() == {"N": 300, "E": 360, "M": 300, "X": 300, "Z": 0}
    assert len(p.inputs) == 12 and p.max_live() == 13
    wl, sets = W.ansatz(batch=3)
    assert wl.pattern.n_meas() == 400 and sets.shape == (3, 400)
    assert wl.pattern.max_live() == 17


def test_batched_widths_and_budgets():
    ws = [W.batched_random(i).meta["width"] for i in range(64)]
    assert min(ws) >= 8 and max(ws) <= 20
    for i in range(8):
        wl = W.batched_random(i)
        assert wl.pattern.max_live() == wl.meta["width"]


def test_seeded_reproducibility():
    a, b = W.plain_small(index=5), W.plain_small(index=5)
    assert a.pattern.cmds == b.pattern.cmds and (a.outcomes == b.outcomes).all()
    c = W.plain_small(index=6)
    assert a.pattern.cmds != c.pattern.cmds


def test_text_round_trip():
    for wl in (W.plain_small(), W.cluster(rows=3, cols=4)):
        t = wl.pattern.to_text()
        q = W.Pattern.from_text(t)
        assert q.cmds == wl.pattern.cmds and q.inputs == wl.pattern.inputs and q.outputs == wl.pattern.outputs


def test_inverse_circuit_is_identity():
    wl = W.plain_large(n_logical=6, n_j=50, n_cz=10)
    g = wl.meta["gates"]
    x = wl.input_state.astype(np.complex128)
    y = ref.circuit_state(6, g + W.inverse_jcz_gates(g), x)
    np.testing.assert_allclose(y, x, atol=1e-12)
