"""CPU checks of the sub-state executor's plan (OWQS_EXEC_SUBSTATES, Sec.
4.1) on a host-only context: the widest sub-state of the library's plan
equals the sub-state oracle's (or one less, where a window is fused), patterns whose components stay apart plan
beyond OWQS_MAX_WIDTH in total, and the entry points that do not run
sub-states refuse them.  No kernel runs here."""
import ctypes

import numpy as np
import pytest

import owqs_workloads as W
from oracle import substates as so

owqs = pytest.importorskip("paper_1604_05659_amd", reason="libowqs.so not built")


@pytest.fixture(scope="module")
def ctx():
    c = owqs.Context(-1)
    yield c
    c.close()


def test_plan_width_is_the_oracles_widest_substate(ctx):
    g = np.random.default_rng(4701)
    for _ in range(40):
        pat = W.random_pattern(g)
        p = owqs.Pattern(ctx, pat)
        p.set_exec(owqs.EXEC_SUBSTATES)
        width, nsteps, _ = p.plan_info()
        inp = W.gaussian_state(len(pat.inputs), g).astype(np.complex128) if pat.inputs else None
        st, _ = so.run(pat, np.zeros(pat.n_meas(), np.uint8), [(list(pat.inputs), inp)] if pat.inputs else None,
                       mode=so.MODE_EOWQS)
        # a fused window (N w; E's; M v) replaces v by w in place, so the
        # plan can be one narrower than the oracle's command-by-command widest
        assert max(st.widest, 1) - 1 <= width <= max(st.widest, 1)
        assert width <= max(pat.max_live(), 1)
        p.close()


def test_separate_components_plan_beyond_the_width_limit(ctx):
    g = np.random.default_rng(4702)
    parts = [W.circuit_to_pattern(12, W.random_jcz_circuit(12, 30, 8, g)) for _ in range(3)]
    pat = W.disjoint_union(parts)
    assert pat.max_live() > owqs.MAX_WIDTH
    p = owqs.Pattern(ctx, pat)
    with pytest.raises(owqs.OwqsError) as e:
        p.plan_info()
    assert e.value.status == owqs.E_WIDTH
    p.set_exec(owqs.EXEC_SUBSTATES)
    with pytest.raises(owqs.OwqsError):   # all 36 inputs as one sub-state
        p.plan_info()
    p.set_input_factors([12, 12, 12])
    width, _, _ = p.plan_info()
    assert max(x.max_live() for x in parts) - 1 <= width <= max(x.max_live() for x in parts)
    p.set_exec(owqs.EXEC_FUSED)
    with pytest.raises(owqs.OwqsError):
        p.plan_info()
    p.close()


def test_other_entry_points_refuse_substates(ctx):
    p = owqs.Pattern(ctx, W.plain_small().pattern)
    p.set_exec(owqs.EXEC_SUBSTATES)
    lib = owqs._lib
    dummy = ctypes.c_void_p(16)  # never dereferenced: the call returns first
    assert lib.owqs_run_basis(p._h, 0, 1, dummy, None, None) == owqs.E_STATE
    assert lib.owqs_run_states(p._h, dummy, 1, dummy, None, None) == owqs.E_STATE
    assert lib.owqs_run_range(p._h, None, 1, 1, 0, 1, None) == owqs.E_STATE
    assert lib.owqs_tune(p._h, None, 1, 1, None, None, None) == owqs.E_STATE
    a = np.zeros(p.n_meas)
    loss = np.zeros(1)
    grad = np.zeros(p.n_meas)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.owqs_adjoint(p._h, None, a.ctypes.data_as(dp), 1, None, 0, loss.ctypes.data_as(dp),
                            grad.ctypes.data_as(dp), 0, None) == owqs.E_STATE
    # reading sub-states needs a sub-state run
    assert lib.owqs_read_substates(p._h, None, 0, None, None, 0, None, None, None, None) == owqs.E_STATE
    # input factors need the sub-state executor
    p.set_exec(owqs.EXEC_FUSED)
    assert lib.owqs_run_factors(p._h, None, None, 0, 1, None) == owqs.E_STATE
    p.close()
