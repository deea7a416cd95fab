"""Host rules of composed window runs in the fused plan (no GPU): every
window of the tile passes is applied either alone or inside exactly one
composed 2x2 map, and maps appear only where a forced run sums no window
(OWQS passes of p = 1/2 windows, EOWQS without the check)."""
import pytest

import owqs_workloads as W

owqs = pytest.importorskip("paper_1604_05659_amd")


@pytest.fixture(scope="module")
def host_ctx():
    return owqs.Context(-1)


def _work(ctx, wl, mode, exec_=owqs.EXEC_FUSED, sum_all=False, bits=12):
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(mode)
    p.set_exec(exec_)
    p.set_outcomes(wl.outcomes)
    p.set_tile_bits(bits)
    if sum_all:
        p.set_sum_all(True)
    r = p.plan_tile_work()
    p.close()
    return r


@pytest.mark.parametrize("bits", [10, 12])
def test_every_window_once(host_ctx, bits):
    wl = W.plain_large(n_logical=18, n_j=400, n_cz=60)
    alone, maps, inside = _work(host_ctx, wl, owqs.MODE_OWQS, bits=bits)
    assert maps > 0 and inside > maps  # some maps compose several windows
    assert alone + inside <= 400  # the circuit's 400 J windows, most of them in tile passes
    assert alone + inside >= 360
    # with every window summed nothing composes (such plans group at most 32
    # windows a pass, so their tile passes may hold a different count)
    total, m2, c2 = _work(host_ctx, wl, owqs.MODE_OWQS, sum_all=True, bits=bits)
    assert (m2, c2) == (0, 0) and 360 <= total <= 400
    # EOWQS sums no window and composes; the check mode groups the same
    # passes (at most 32 windows each in both) and sums every window
    ea, em, ei = _work(host_ctx, wl, owqs.MODE_EOWQS, bits=bits)
    assert em > 0 and ei > em
    assert _work(host_ctx, wl, owqs.MODE_EOWQS_CHECK, bits=bits) == (ea + ei, 0, 0)


def test_plain_plan_has_no_tile_work(host_ctx):
    wl = W.plain_large(n_logical=18, n_j=100, n_cz=20)
    assert _work(host_ctx, wl, owqs.MODE_OWQS, exec_=owqs.EXEC_PLAIN) == (0, 0, 0)


def test_cz_on_every_wire_between_windows_stops_composition(host_ctx):
    """J, CZ on the same wire, J, ...: each window meets an E on its own bit
    before the next one, so every map holds one window (the rounds still
    run maps only: all or nothing per pass)."""
    n = 16
    gates = []
    for r in range(6):
        for q in range(n):
            gates.append(("J", q, 0.3 + 0.1 * q + r))
        for q in range(n):
            gates.append(("CZ", q, (q + 1) % n))
    pat = W.circuit_to_pattern(n, gates)
    wl = W.Workload(pat, W.outcome_bits(pat.n_meas(), W.rng(9, W.P_OUTCOME, 0)),
                    W.gaussian_state(n, W.rng(9, W.P_INPUT, 0)), {})
    alone, maps, inside = _work(host_ctx, wl, owqs.MODE_OWQS)
    assert maps > 0 and inside == maps


def test_substate_passes_compose(host_ctx):
    """Sub-state plans (three 16-qubit circuits side by side) compose the
    windows of their tile passes the same way."""
    import numpy as np
    g = np.random.default_rng([160405659, 9, 0])
    parts = [W.circuit_to_pattern(16, W.random_jcz_circuit(16, 400, 60, g)) for _ in range(3)]
    q = owqs.Pattern(host_ctx, W.disjoint_union(parts))
    q.set_exec(owqs.EXEC_SUBSTATES)
    q.set_input_factors([16, 16, 16])
    alone, maps, inside = q.plan_tile_work()
    assert maps > 0 and inside > maps, (alone, maps, inside)
    assert alone + inside <= 3 * 400
    q.set_sum_all(True)
    assert q.plan_tile_work()[1:] == (0, 0)
    q.close()
