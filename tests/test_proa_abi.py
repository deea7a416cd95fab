"""CPU checks of the library's pattern reordering (owqs_pattern_reorder,
PROA, Sec. 4.3) against the reordering oracle: the same measurement order,
the same commands, the same largest state-space, on Table I, clusters and
random standard-form patterns; plus the command read-back
(owqs_pattern_commands) and the argument checks.  Host-only context."""
import json
import os

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc
from oracle import proa

owqs = pytest.importorskip("paper_1604_05659_amd", reason="libowqs.so not built")

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    c = owqs.Context(-1)
    yield c
    c.close()


def canon(cmds):
    out = []
    for c in cmds:
        if c[0] == "N":
            out.append(("N", int(c[1])))
        elif c[0] == "E":
            out.append(("E", int(c[1]), int(c[2])))
        elif c[0] == "M":
            out.append(("M", int(c[1]), float(c[2]), tuple(int(q) for q in c[3]), tuple(int(q) for q in c[4])))
        else:
            out.append((c[0], int(c[1]), tuple(int(q) for q in c[2])))
    return out


def table1_pattern():
    g = json.load(open(os.path.join(GOLD, "table1_swap_proa.json")))
    cmds = [("N", q) for q in g["qubits"]] + [("E", a, b) for a, b in g["edges"]]
    cmds += [("M", q, 0.0, (), ()) for q in g["qubits"] if q not in g["outputs"]]
    return g, W.Pattern([], g["outputs"], cmds)


def check_against_oracle(ctx, pat, free=False, weights=None):
    lib_pat = owqs.Pattern(ctx, pat)
    re_lib, stats = lib_pat.reorder(weights=weights, ignore_dependencies=free)
    order, spaces, m, alpha = proa.proa(pat, weights=weights, ignore_dependencies=free)
    want = proa.reordered_pattern(pat, order, positive_branch=free)
    got = re_lib.commands()
    assert [c[1] for c in got.cmds if c[0] == "M"] == order
    assert canon(got.cmds) == canon(want.cmds)
    assert got.inputs == list(pat.inputs) and got.outputs == list(pat.outputs)
    assert stats["max_state_space"] == m
    assert stats["alpha"] == alpha
    assert stats["max_live"] == re_lib.max_live == W.Pattern(got.inputs, got.outputs, got.cmds).max_live()
    re_lib.close()
    lib_pat.close()
    return got, stats


def test_commands_read_back_what_was_loaded(ctx):
    g = np.random.default_rng(4401)
    for _ in range(10):
        pat = W.random_pattern(g)
        p = owqs.Pattern(ctx, pat)
        got = p.commands()
        assert canon(got.cmds) == canon(pat.cmds)
        assert got.inputs == list(pat.inputs) and got.outputs == list(pat.outputs)
        # angles set later are the ones read back
        a = np.linspace(0.1, 1.0, p.n_meas)
        p.set_angles(a)
        assert [c[2] for c in p.commands().cmds if c[0] == "M"] == list(a)
        p.close()


def test_table1_order_through_the_abi(ctx):
    g, pat = table1_pattern()
    got, stats = check_against_oracle(ctx, pat)
    assert [c[1] for c in got.cmds if c[0] == "M"] == g["order"]
    assert stats["max_state_space"] == 3


@pytest.mark.parametrize("free", [False, True])
def test_random_standard_patterns_match_the_oracle(ctx, free):
    g = np.random.default_rng(4402 + free)
    for _ in range(40):
        pat = W.random_standard_pattern(g, n_qubits=int(g.integers(4, 14)), n_in=int(g.integers(0, 3)),
                                        n_out=int(g.integers(1, 4)), extra_edges=int(g.integers(0, 8)),
                                        max_dom=int(g.integers(0, 4)))
        check_against_oracle(ctx, pat, free=free)


def test_explicit_weights_match_the_oracle(ctx):
    g = np.random.default_rng(4404)
    for w in [(1.0, 0.0, 0.0, 1.0), (2.0, 3.0, 0.5, 1.0), (1.0, 1.0, 2.0, 4.0)]:
        for _ in range(8):
            pat = W.random_standard_pattern(g, n_qubits=10, n_in=1, n_out=2, extra_edges=5)
            check_against_oracle(ctx, pat, weights=w)


def test_cluster_order_matches_the_oracle_and_the_bound(ctx):
    for rows, cols in [(3, 5), (4, 9), (5, 12)]:
        std = W.standard_form(W.cluster(rows=rows, cols=cols).pattern)
        _, stats = check_against_oracle(ctx, std)
        assert stats["max_state_space"] == rows + 1
        # one vector holds every prepared, unmeasured qubit: the rows of the
        # current column and the next one's first qubit, plus v itself
        assert stats["max_live"] <= rows + 2


def test_reordered_pattern_computes_the_source(ctx):
    """The library's reordered pattern, run by the oracle, gives the source
    pattern's output and joint outcome probability (Sec. 4.3 Proposition)."""
    g = np.random.default_rng(4405)
    for _ in range(10):
        pat = W.random_standard_pattern(g, n_qubits=9, n_in=2, n_out=2, extra_edges=4)
        p = owqs.Pattern(ctx, pat)
        re, _ = p.reorder()
        spec = re.commands()
        rp = W.Pattern(spec.inputs, spec.outputs, spec.cmds)
        per_q = {c[1]: int(g.integers(2)) for c in pat.cmds if c[0] == "M"}
        oc_src = np.array([per_q[c[1]] for c in pat.cmds if c[0] == "M"], np.uint8)
        oc_re = np.array([per_q[c[1]] for c in rp.cmds if c[0] == "M"], np.uint8)
        inp = W.gaussian_state(2, g).astype(np.complex128)
        want, pw = oc.run(pat, oc_src, inp)
        got, pg = oc.run(rp, oc_re, inp)
        np.testing.assert_allclose(got, want, atol=1e-10)
        assert float(np.prod(pg)) == pytest.approx(float(np.prod(pw)), rel=1e-9)
        re.close()
        p.close()


def test_repeated_e_cancels(ctx):
    pat = W.Pattern([0], [2], [("N", 1), ("N", 2), ("E", 0, 1), ("E", 1, 2), ("E", 0, 2), ("E", 2, 0),
                               ("M", 0, 0.3, (), ()), ("M", 1, 0.7, (0,), ()), ("X", 2, (1,)), ("Z", 2, (0,))])
    got, _ = check_against_oracle(ctx, pat)
    assert ("E", 0, 2) not in canon(got.cmds) and ("E", 2, 0) not in canon(got.cmds)


def test_reorder_argument_checks(ctx):
    # a correction before an E it does not commute with: not standard form
    bad = W.Pattern([0], [2], [("N", 1), ("N", 2), ("E", 0, 1), ("M", 0, 0.0, (), ()), ("X", 1, (0,)),
                               ("E", 1, 2), ("M", 1, 0.0, (), ())])
    p = owqs.Pattern(ctx, bad)
    with pytest.raises(owqs.OwqsError) as e:
        p.reorder()
    assert e.value.status == owqs.E_PATTERN
    p.close()
    ok = owqs.Pattern(ctx, table1_pattern()[1])
    with pytest.raises(owqs.OwqsError) as e:
        ok.reorder(weights=(1.0, -1.0, 0.5, 1.0))
    assert e.value.status == owqs.E_INVALID_ARG
    ok.close()


def test_no_measurements(ctx):
    pat = W.Pattern([0, 1], [0, 1], [("E", 0, 1)])
    got, stats = check_against_oracle(ctx, pat)
    assert canon(got.cmds) == [("E", 0, 1)] and stats["max_state_space"] == 0


def test_table3_cnot(ctx):
    """Table III, CNOT row: m = 3 in both modes, through the library."""
    pat = W.Pattern([1, 2], [1, 4], [("N", 3), ("N", 4), ("E", 1, 3), ("E", 2, 3), ("E", 3, 4),
                                     ("M", 2, 0.0, (), ()), ("M", 3, 0.0, (), ()),
                                     ("X", 4, (3,)), ("Z", 4, (2,)), ("Z", 1, (2,))])
    for free in (False, True):
        _, stats = check_against_oracle(ctx, pat, free=free)
        assert stats["max_state_space"] == 3
