"""CPU checks of the C ABI: the library loads, exports every function that
include/owqs.h declares, and validates patterns on a host-only context
(device -1).  No kernel runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

import owqs_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "owqs.h")

owqs = pytest.importorskip("paper_1604_05659_amd", reason="libowqs.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(owqs_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(owqs.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # and the binding wraps each of them
    assert set(names) == set(owqs.EXPORTED)


def test_cmd_struct_layout_matches_header():
    assert ctypes.sizeof(owqs.OwqsCmd) == 40
    assert owqs.OwqsCmd.angle.offset == 32


@pytest.fixture(scope="module")
def host_ctx():
    return owqs.Context(-1)


def test_status_strings():
    assert owqs._lib.owqs_status_str(0) == b"OWQS_OK"
    assert owqs._lib.owqs_status_str(-3) == b"OWQS_E_ZERO_PROB"


def test_info_matches_structure(host_ctx):
    for wl in (W.plain_small(), W.cluster(rows=4, cols=6), W.recognition(n_logical=5, n_j=30, n_cz=6)):
        p = owqs.Pattern(host_ctx, wl.pattern)
        assert p.n_meas == wl.pattern.n_meas()
        assert p.max_live == wl.pattern.max_live()
        assert p.n_in == len(wl.pattern.inputs)
        assert p.n_out == len(wl.pattern.outputs)
        assert p.ncmds == len(wl.pattern.cmds)


def test_text_format_round_trip(host_ctx):
    wl = W.cluster(rows=3, cols=5)
    text = wl.pattern.to_text()
    a = owqs.Pattern(host_ctx, wl.pattern)
    b = owqs.Pattern(host_ctx, text=text)
    assert (a.n_meas, a.max_live, a.n_in, a.n_out, a.ncmds) == (b.n_meas, b.max_live, b.n_in, b.n_out, b.ncmds)
    with pytest.raises(owqs.OwqsError) as e:
        owqs.Pattern(host_ctx, text="inputs 0\noutputs 1\nQ 3\n")
    assert e.value.status == owqs.E_INVALID_ARG


@pytest.mark.parametrize("cmds,ins,outs", [
    ([("M", 2, 0.0, (), ())], [1], [2]),                                  # D2
    ([("M", 1, 0.0, (), ()), ("M", 1, 0.0, (), ())], [1], []),            # D1
    ([("N", 2), ("M", 1, 0.0, (), ()), ("E", 1, 2)], [1], [2]),           # D1
    ([("M", 1, 0.0, (), ())], [1], [1]),                                  # D3
    ([("N", 2), ("M", 1, 0.0, (3,), ())], [1], [2]),                      # D0
    ([("N", 2), ("N", 2)], [1], [1, 2]),                                  # D2
    ([("N", 2)], [1], [1]),                                               # D3
    ([("N", 2), ("X", 2, (5,)), ("M", 1, 0.0, (), ())], [1], [2]),        # D0
])
def test_rule_violations_rejected(host_ctx, cmds, ins, outs):
    with pytest.raises(owqs.OwqsError) as e:
        owqs.Pattern(host_ctx, W.Pattern(ins, outs, cmds))
    assert e.value.status == owqs.E_PATTERN


def test_width_limit_and_bad_arguments(host_ctx):
    n = 36
    cmds = [("N", q) for q in range(n)] + [("M", q, 0.0, (), ()) for q in range(n - 1)]
    wide = owqs.Pattern(host_ctx, W.Pattern([], [n - 1], cmds))  # loads: it can still be reordered
    assert wide.max_live == n
    with pytest.raises(owqs.OwqsError) as e:
        wide.plan_info()
    assert e.value.status == owqs.E_WIDTH
    narrow, stats = wide.reorder()
    assert stats["max_live"] == narrow.max_live == 1  # no E: one qubit at a time
    narrow.close()
    wide.close()
    p = owqs.Pattern(host_ctx, W.plain_small().pattern)
    with pytest.raises(owqs.OwqsError):
        p.set_outcomes(np.zeros(3, np.uint8))
    with pytest.raises(owqs.OwqsError):
        p.set_outcomes(np.full(p.n_meas, 2, np.uint8))
    with pytest.raises(owqs.OwqsError):
        p.set_angles(np.zeros(p.n_meas + 1))
    with pytest.raises(owqs.OwqsError) as e:
        p.set_mode(7)
    # a host-only context cannot run
    st = owqs._lib.owqs_run(p._h, None, 1, 1, None)
    assert st == owqs.E_STATE


def test_random_patterns_validate(host_ctx):
    g = np.random.default_rng(99)
    for _ in range(50):
        pat = W.random_pattern(g)
        p = owqs.Pattern(host_ctx, pat)
        assert p.max_live == pat.max_live()


def test_single_hip_runtime_in_process():
    """The binding loads PyTorch's HIP runtime before libowqs, so only one copy
    of libamdhip64 is mapped (two copies break device-pointer sharing)."""
    maps = open("/proc/self/maps").read()
    libs = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(libs) == 1, libs


def test_fused_plan_forms_windows(host_ctx):
    """The fused plan turns N w; E...; M v; corrections into one step: the
    J/CZ translations keep only windows and CZ steps, the cluster's
    N, E, E, M groups become windows too."""
    wl = W.plain_large(n_logical=10, n_j=100, n_cz=20)
    p = owqs.Pattern(host_ctx, wl.pattern)
    p.set_exec(owqs.EXEC_FUSED)
    w, n, _ = p.plan_info()
    assert n == 100 + 20 and w == 10
    p.set_exec(owqs.EXEC_PLAIN)
    w2, n2, _ = p.plan_info()
    assert w2 == 11 and n2 == 100 * 3 + 20  # N, E, M per J (X only when its signal is 1) + CZ
    wl = W.cluster(rows=20, cols=200)
    q = owqs.Pattern(host_ctx, wl.pattern)
    q.set_outcomes(wl.outcomes)
    q.set_exec(owqs.EXEC_FUSED)
    w3, n3, x3 = q.plan_info()
    assert w3 <= 21 and n3 < 4400, n3
    assert x3 < n3  # runs of windows group into tile passes at width >= 18


def test_tile_grouping_looks_ahead(host_ctx):
    """Host plan of the large circuit (24 logical qubits, 2000 J + 300 CZ):
    a step whose slot does not fit the tile no longer ends the pass, so the
    2300 steps go into about 22 passes in OWQS mode (at most 128 windows
    with p = 1/2 a pass; the tile's free slots end most passes first) and 64
    in EOWQS mode (at most 32); the sub-state plan of three 16-qubit
    circuits groups each sub-state's steps the same way."""
    wl = W.plain_large()
    p = owqs.Pattern(host_ctx, wl.pattern)
    p.set_outcomes(wl.outcomes)
    p.set_exec(owqs.EXEC_FUSED)
    for mode, most in ((owqs.MODE_OWQS, 50), (owqs.MODE_EOWQS, 70)):  # EOWQS: 32 windows a pass
        p.set_mode(mode)
        w, n, passes = p.plan_info()
        assert (w, n) == (24, 2300)
        assert 2000 / (128 if mode == owqs.MODE_OWQS else 32) <= passes <= most, (mode, passes)
    g = np.random.default_rng([160405659, 9, 0])
    parts = [W.circuit_to_pattern(16, W.random_jcz_circuit(16, 400, 60, g)) for _ in range(3)]
    q = owqs.Pattern(host_ctx, W.disjoint_union(parts))
    q.set_exec(owqs.EXEC_SUBSTATES)
    q.set_input_factors([16, 16, 16])
    w, n, launches = q.plan_info()
    assert w == 16 and n == 1380 and launches <= 120, (w, n, launches)


def test_outcome_seed_follows_the_oracle_stream(host_ctx):
    from oracle import core as oc
    for wl in (W.plain_small(), W.cluster(rows=4, cols=6)):
        p = owqs.Pattern(host_ctx, wl.pattern)
        for seed in (0, 1, 1234567, 2**64 - 1, 160405659):
            p.set_outcome_seed(seed)
            np.testing.assert_array_equal(p.outcomes(), oc.outcomes_from_seed(seed, p.n_meas))
        p.set_outcomes(wl.outcomes)
        np.testing.assert_array_equal(p.outcomes(), wl.outcomes)
        p.close()


def test_ranged_run_argument_checks(host_ctx):
    p = owqs.Pattern(host_ctx, W.plain_small().pattern)
    # no ranged run to read yet
    st = owqs._lib.owqs_read_live(p._h, None, 0, None, None, None)
    assert st == owqs.E_STATE
    # a range outside the pattern is rejected before anything else
    assert owqs._lib.owqs_run_range(p._h, None, 1, 1, 3, 2, None) == owqs.E_INVALID_ARG
    assert owqs._lib.owqs_run_range(p._h, None, 1, 1, 0, p.ncmds + 1, None) == owqs.E_INVALID_ARG
    # a host-only context cannot run
    assert owqs._lib.owqs_run_range(p._h, None, 1, 1, 0, 4, None) == owqs.E_STATE
    p.close()


def test_uniforms_argument_checks(host_ctx):
    wl = W.plain_small()
    p = owqs.Pattern(host_ctx, wl.pattern)
    with pytest.raises(owqs.OwqsError):
        p.set_uniforms(np.full(p.n_meas - 1, 0.5))
    for bad in (1.0, -0.1, float("nan")):
        u = np.full(p.n_meas, 0.5)
        u[3] = bad
        with pytest.raises(owqs.OwqsError):
            p.set_uniforms(u)
    p.set_uniforms(np.full(p.n_meas, 0.25))
    p.set_uniforms(None)
    # before any run, the outcomes read back are the forced ones
    p.set_outcomes(wl.outcomes)
    np.testing.assert_array_equal(p.read_outcomes(), wl.outcomes)
    p.close()


def test_noalloc_rejects_width_and_host_context(host_ctx):
    """owqs_run_noalloc checks the live width against its fixed array before
    anything else (a clear OWQS_E_WIDTH), and a host-only context cannot run."""
    wide = W.plain_large(n_logical=owqs.NOALLOC_MAX_WIDTH, n_j=4, n_cz=1)   # live width 23
    p = owqs.Pattern(host_ctx, wide.pattern)
    assert p.max_live == owqs.NOALLOC_MAX_WIDTH + 1
    st = owqs._lib.owqs_run_noalloc(p._h, None, 1 << p.n_in, None, 1 << p.n_out, None, None, None)
    assert st == owqs.E_WIDTH
    assert b"allocation-free limit 22" in owqs._lib.owqs_last_error(host_ctx._h)
    ok = W.plain_small()
    q = owqs.Pattern(host_ctx, ok.pattern)
    st = owqs._lib.owqs_run_noalloc(q._h, None, 1, None, 1 << q.n_out, None, None, None)
    assert st == owqs.E_INVALID_ARG          # no output buffer
    st = owqs._lib.owqs_run_noalloc(q._h, None, 1, 1234, 1 << q.n_out, None, None, None)
    assert st == owqs.E_STATE                # host-only context
    p.close()
    q.close()
