"""GPU parity of the sub-state executor (OWQS_EXEC_SUBSTATES, Sec. 4.1,
Sec. 4.4.1) against the sub-state oracle: the assembled output, the
probabilities, and each factor (which qubits, and its amplitudes) with the
scalar of the fully measured sub-states; Fig. 8 with two one-qubit input
sub-states; patterns of separate components wider than OWQS_MAX_WIDTH in
total; tensor-product merges of large sub-states; PROA's order of the 20x200
cluster.  Bar: 1e-5 on complex64 amplitudes, 1e-5 on FP64 probabilities."""
import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc
from oracle import substates as so

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-5
P_TOL = 1e-5

torch = pytest.importorskip("torch")
owqs = pytest.importorskip("paper_1604_05659_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return owqs.Context(0)


def cuda(v):
    return torch.as_tensor(np.asarray(v, np.complex64)).cuda()


def run_sub(ctx, pat, outcomes, factors, mode=owqs.MODE_OWQS, graph=True):
    """factors: [(qubits, vector)] covering the inputs in input order."""
    p = owqs.Pattern(ctx, pat)
    p.set_exec(owqs.EXEC_SUBSTATES)
    p.set_mode(mode)
    p.set_graph(graph)
    p.set_outcomes(np.asarray(outcomes, np.uint8))
    p.run_factors([cuda(v) for _, v in factors])
    torch.cuda.synchronize()
    return p


def compare_factors(p, st, pat):
    """Library factors against the oracle's sub-states (both hold only outputs)."""
    got, scalar = p.read_substates()
    want = {tuple(sorted(qs)): (qs, vec) for qs, vec in st.subs}
    assert {tuple(sorted(q)) for q, _ in got} == set(want)
    pos = {q: k for k, q in enumerate(pat.outputs)}
    for qs, vec in got:
        assert qs == sorted(qs, key=lambda q: pos[q])   # outputs order inside a factor
        oq, ov = want[tuple(sorted(qs))]
        ref = so.factor_in_order(oq, ov, qs)
        assert np.max(np.abs(vec.astype(np.complex128) - ref)) <= AMP_TOL
    assert abs(scalar - st.scalar) <= AMP_TOL
    firsts = [min(pos[q] for q in qs) for qs, _ in got]
    assert firsts == sorted(firsts)


def test_random_patterns_against_the_substate_oracle(ctx):
    g = np.random.default_rng(4801)
    done = 0
    for i in range(120):
        pat = W.random_pattern(g)
        outc = g.integers(0, 2, pat.n_meas()).astype(np.uint8)
        inp = W.gaussian_state(len(pat.inputs), g).astype(np.complex64).astype(np.complex128)
        factors = [(list(pat.inputs), inp)] if pat.inputs else []
        try:
            st, pw = so.run(pat, outc, factors or None)
        except so.SubStateError:
            continue
        if len(pw) and pw.min() < 1e-6:
            continue  # a forced outcome of (almost) zero probability
        print(f"[substates] random {i}", flush=True)
        p = run_sub(ctx, pat, outc, factors)
        got = p.read_state().cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(got - so.assemble(st, pat.outputs))) <= AMP_TOL, i
        np.testing.assert_allclose(p.read_probs(), pw, atol=P_TOL)
        compare_factors(p, st, pat)
        p.close()
        done += 1
    assert done >= 60


@pytest.mark.parametrize("mode", [owqs.MODE_EOWQS, owqs.MODE_EOWQS_CHECK, owqs.MODE_OWQS])
def test_flow_circuits_all_modes(ctx, mode):
    g = np.random.default_rng(4802 + mode)
    for i in range(12):
        nl = int(g.integers(2, 7))
        pat = W.circuit_to_pattern(nl, W.random_jcz_circuit(nl, int(g.integers(5, 40)), int(g.integers(1, 8)), g))
        outc = g.integers(0, 2, pat.n_meas()).astype(np.uint8)
        # every input its own sub-state
        vecs = [W.gaussian_state(1, g).astype(np.complex64).astype(np.complex128) for _ in pat.inputs]
        factors = [([q], v) for q, v in zip(pat.inputs, vecs)]
        st, pw = so.run(pat, outc, factors, mode=so.MODE_OWQS if mode == owqs.MODE_OWQS else so.MODE_EOWQS)
        p = run_sub(ctx, pat, outc, factors, mode)
        got = p.read_state().cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(got - so.assemble(st, pat.outputs))) <= AMP_TOL, (mode, i)
        compare_factors(p, st, pat)
        if mode != owqs.MODE_EOWQS:
            np.testing.assert_allclose(p.read_probs(), 0.5, atol=P_TOL)
        p.close()


def test_fig8_with_one_qubit_input_substates(ctx):
    """Fig. 8: the CNOT of Eq. 23 on |q2 q1> = |11>, inputs as two one-qubit
    sub-states; the result is the printed stage (f), |q4 q1> = |01>."""
    cmds = [("N", 3), ("N", 4), ("E", 2, 3), ("M", 2, 0.0, (), ()), ("E", 3, 4), ("E", 1, 3),
            ("M", 3, 0.0, (), ()), ("Z", 1, (2,)), ("Z", 4, (2,)), ("X", 4, (3,))]
    pat = W.Pattern([1, 2], [1, 4], cmds)
    one = np.array([0, 1.0])
    p = run_sub(ctx, pat, [0, 1], [([1], one), ([2], one)])
    (qs, vec), = p.read_substates()[0]
    assert qs == [1, 4]
    # printed (0 1 0 0) over |q4 q1>, most significant first: q1 = 1, q4 = 0
    np.testing.assert_allclose(vec, [0, 1, 0, 0], atol=1e-6)
    np.testing.assert_allclose(p.read_probs(), [0.5, 0.5], atol=1e-7)
    p.close()


def test_separate_components_beyond_the_width_limit(ctx):
    """Three 12-qubit circuits side by side: 36 inputs, 36 outputs and a live
    width above OWQS_MAX_WIDTH as one vector; as sub-states each factor is its
    circuit's output, against the elimination oracle per circuit."""
    g = np.random.default_rng(4803)
    parts = [W.circuit_to_pattern(12, W.random_jcz_circuit(12, 40, 10, g)) for _ in range(3)]
    pat = W.disjoint_union(parts)
    assert pat.max_live() > owqs.MAX_WIDTH
    outs = [g.integers(0, 2, x.n_meas()).astype(np.uint8) for x in parts]
    ins = [W.gaussian_state(12, g).astype(np.complex64).astype(np.complex128) for _ in parts]
    # measurement order of the union: interleaved like its commands
    per_q = {}
    for k, (x, o) in enumerate(zip(parts, outs)):
        for c, b in zip([c for c in x.cmds if c[0] == "M"], o):
            per_q[c[1] + 1000 * k] = int(b)
    outc = np.array([per_q[c[1]] for c in pat.cmds if c[0] == "M"], np.uint8)
    p = owqs.Pattern(ctx, pat)
    p.set_exec(owqs.EXEC_SUBSTATES)
    p.set_outcomes(outc)
    p.run_factors([cuda(v) for v in ins])
    assert p.plan_info()[0] <= max(x.max_live() for x in parts)
    got, scalar = p.read_substates()
    assert len(got) == 3 and abs(abs(scalar) - 1) < 1e-6
    for k, (x, o, v) in enumerate(zip(parts, outs, ins)):
        want, _ = oc.run(x, o, v)
        qs, vec = got[k]
        assert qs == [q + 1000 * k for q in x.outputs]
        # the global phase of the scalar belongs to the product, not to one factor
        assert np.max(np.abs(vec * (scalar if k == 0 else 1) - want)) <= AMP_TOL
    buf = torch.empty(1, dtype=torch.complex64, device="cuda")
    assert owqs._lib.owqs_read_state(p._h, buf.data_ptr(), 1, 1, None) == owqs.E_WIDTH  # 2^36 outputs
    p.close()


@pytest.mark.parametrize("na,nb", [(11, 11), (12, 9), (6, 14)])
def test_large_tensor_product_merge(ctx, na, nb):
    """Two circuits that finish apart, then an E between outputs of each:
    one tensor-product merge of 2^na by 2^nb amplitudes, against the
    elimination oracle (one vector)."""
    g = np.random.default_rng(4804 + na)
    pa = W.circuit_to_pattern(na, W.random_jcz_circuit(na, 3 * na, na, g))
    pb = W.circuit_to_pattern(nb, W.random_jcz_circuit(nb, 3 * nb, nb, g))
    both = W.disjoint_union([pa, pb])
    cmds = list(both.cmds) + [("E", both.outputs[0], both.outputs[-1])]
    pat = W.Pattern(both.inputs, both.outputs, cmds)
    outc = g.integers(0, 2, pat.n_meas()).astype(np.uint8)
    va = W.gaussian_state(na, g).astype(np.complex64).astype(np.complex128)
    vb = W.gaussian_state(nb, g).astype(np.complex64).astype(np.complex128)
    want, pw = oc.run(pat, outc, np.kron(vb, va))
    print(f"[substates] merge {na}x{nb}", flush=True)
    p = run_sub(ctx, pat, outc, [(pa.inputs, va), (pb.inputs, vb)])
    got = p.read_state().cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - want)) <= AMP_TOL
    np.testing.assert_allclose(p.read_probs(), pw, atol=P_TOL)
    (qs, vec), = p.read_substates()[0]
    assert qs == list(pat.outputs)
    p.close()


def test_graph_replays_and_eager_agree(ctx):
    g = np.random.default_rng(4805)
    pat = W.circuit_to_pattern(6, W.random_jcz_circuit(6, 40, 10, g))
    p = owqs.Pattern(ctx, pat)
    p.set_exec(owqs.EXEC_SUBSTATES)
    for r in range(4):
        outc = g.integers(0, 2, pat.n_meas()).astype(np.uint8)
        inp = W.gaussian_state(6, g).astype(np.complex64)
        p.set_outcomes(outc)
        p.set_graph(r % 2 == 0)
        p.run(cuda(inp))
        got = p.read_state().cpu().numpy().astype(np.complex128)
        torch.cuda.synchronize()
        want, _ = oc.run(pat, outc, inp.astype(np.complex128))
        assert np.max(np.abs(got - want)) <= AMP_TOL, r
    p.close()


def test_proa_order_of_the_cluster_as_substates(ctx):
    """The 20 x 200 cluster in standard form, reordered by the library, run as
    sub-states: equal to the fused single-vector run of the same order."""
    wl = W.cluster(rows=20, cols=200)
    src = owqs.Pattern(ctx, W.standard_form(wl.pattern))
    re, stats = src.reorder()
    spec = re.commands()
    per_q = dict(zip([c[1] for c in wl.pattern.cmds if c[0] == "M"], (int(b) for b in wl.outcomes)))
    outc = np.array([per_q[c[1]] for c in spec.cmds if c[0] == "M"], np.uint8)
    re.set_outcomes(outc)
    re.set_exec(owqs.EXEC_FUSED)
    re.run(None)
    want = re.read_state().cpu().numpy().astype(np.complex128)
    re.set_exec(owqs.EXEC_SUBSTATES)
    assert re.plan_info()[0] in (stats["max_state_space"] - 1, stats["max_state_space"])  # a fused window is one narrower
    re.run(None)
    got = re.read_state().cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - want)) <= AMP_TOL
    re.close()
    src.close()


@pytest.mark.parametrize("na,nb", [(6, 6), (13, 13), (20, 2), (19, 3)])
def test_profiled_run_times_every_step(ctx, na, nb):
    """Two path graph states merged by one E (both merge kernels: A below and
    above 2^20 amplitudes): the profiled run reports one merge
    (8 (2^a + 2^b + 2^(a+b)) bytes) and the state equals the oracle's."""
    cmds = []
    for base, n in ((0, na), (100, nb)):
        for k in range(n):
            cmds.append(("N", base + k))
            if k:
                cmds.append(("E", base + k - 1, base + k))
    cmds.append(("E", na // 2, 100))
    pat = W.Pattern([], list(range(na)) + [100 + k for k in range(nb)], cmds)
    st, _ = so.run(pat, [], None)
    p = owqs.Pattern(ctx, pat)
    p.set_exec(owqs.EXEC_SUBSTATES)
    prof = p.run_profiled(None)
    assert prof["kron(merge)"]["launches"] == 1
    assert prof["kron(merge)"]["bytes"] == 8 * (2 ** na + 2 ** nb + 2 ** (na + nb))
    assert prof["prepare(N)"]["launches"] == na + nb
    got = p.read_state().cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - so.assemble(st, pat.outputs))) <= AMP_TOL
    p.close()


@pytest.mark.parametrize("case", ["identity", "permuted", "all_measured", "fresh_outputs", "empty"])
def test_degenerate_patterns(ctx, case):
    """No commands (the input factors are the output, in output order), every
    qubit measured (one amplitude: the scalar), outputs never entangled
    (one |+> factor each), and the empty pattern (the scalar 1)."""
    g = np.random.default_rng(4901)
    if case == "identity":
        pat, factors, outc = W.Pattern([0, 1, 2], [0, 1, 2], []), [([0, 1], None), ([2], None)], []
    elif case == "permuted":
        pat, factors, outc = W.Pattern([0, 1, 2], [2, 0, 1], []), [([0], None), ([1, 2], None)], []
    elif case == "all_measured":
        pat = W.Pattern([0], [], [("N", 1), ("E", 0, 1), ("M", 0, 0.7, (), ()), ("N", 2), ("M", 1, 1.3, (0,), ()),
                                  ("M", 2, 0.2, (), ())])
        factors, outc = [([0], None)], [1, 0, 1]
    elif case == "fresh_outputs":
        pat = W.Pattern([], [3, 4], [("N", 3), ("N", 5), ("N", 4), ("M", 5, 0.4, (), ()), ("Z", 3, (5,))])
        factors, outc = [], [1]
    else:
        pat, factors, outc = W.Pattern([], [], []), [], []
    factors = [(qs, W.gaussian_state(len(qs), g).astype(np.complex64).astype(np.complex128)) for qs, _ in factors]
    st, pw = so.run(pat, outc, factors or None)
    p = run_sub(ctx, pat, outc, factors)
    got = p.read_state().cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - so.assemble(st, pat.outputs))) <= AMP_TOL
    np.testing.assert_allclose(p.read_probs(), pw, atol=P_TOL)
    compare_factors(p, st, pat)
    p.close()


def with_extra_corrections(pat, g, count):
    """The pattern with `count` X/Z commands inserted after random gate ends,
    each on an entangled live qubit, its domain one or two measured qubits
    (standalone corrections inside the tile passes)."""
    live, touched, measured, cmds = set(pat.inputs), set(pat.inputs), [], []
    ends = []
    for k, c in enumerate(pat.cmds):
        nxt = pat.cmds[k + 1] if k + 1 < len(pat.cmds) else None
        if c[0] in ("M", "X", "Z") and not (nxt and nxt[0] in ("X", "Z")) and measured:
            ends.append(k)
        if c[0] == "M":
            measured.append(c[1])
    picks = set(g.choice(ends, size=min(count, len(ends)), replace=False).tolist())
    measured = []
    for k, c in enumerate(pat.cmds):
        cmds.append(c)
        if c[0] == "N":
            live.add(c[1])
        elif c[0] == "E":
            touched.update(c[1:3])
        elif c[0] == "M":
            live.discard(c[1])
            measured.append(c[1])
        if k in picks:
            q = int(g.choice(sorted(live & touched)))
            dom = tuple(int(x) for x in g.choice(measured, size=int(g.integers(1, 3)), replace=False))
            cmds.append(("X" if g.integers(0, 2) else "Z", q, dom))
    return W.Pattern(pat.inputs, pat.outputs, cmds)


@pytest.mark.parametrize("mode", [owqs.MODE_OWQS, owqs.MODE_EOWQS, owqs.MODE_EOWQS_CHECK])
def test_tile_passes_per_substate(ctx, mode):
    """Two circuits of 15 and 16 logical qubits side by side, with extra X/Z
    corrections: each sub-state's windows, E, X and Z at width >= 15 run as
    tile passes (far fewer launches than steps), interleaved with the other
    sub-state's; factors and probabilities against the sub-state oracle,
    with and without graph capture, and the profiled run counts tile passes."""
    g = np.random.default_rng(4810 + mode)
    parts = [with_extra_corrections(W.circuit_to_pattern(nl, W.random_jcz_circuit(nl, 70, 14, g)), g, 12)
             for nl in (15, 16)]
    pat = W.disjoint_union(parts)
    outc = g.integers(0, 2, pat.n_meas()).astype(np.uint8)
    vecs = [W.gaussian_state(len(x.inputs), g).astype(np.complex64).astype(np.complex128) for x in parts]
    factors = [(list(np.array(x.inputs) + 1000 * k), v) for k, (x, v) in enumerate(zip(parts, vecs))]
    st, pw = so.run(pat, outc, factors, mode=so.MODE_OWQS if mode == owqs.MODE_OWQS else so.MODE_EOWQS)
    for graph in (True, False):
        print(f"[substates] tile passes mode {mode} graph {graph}", flush=True)
        p = run_sub(ctx, pat, outc, factors, mode, graph)
        width, nsteps, npasses = p.plan_info()
        assert width == 16 and npasses < nsteps // 4, (width, nsteps, npasses)
        compare_factors(p, st, pat)
        if mode != owqs.MODE_EOWQS:
            np.testing.assert_allclose(p.read_probs(), pw, atol=P_TOL)
        p.check()
        p.close()
    # one circuit, its input as one factor: the profiled run times the passes
    one = parts[1]
    o1 = g.integers(0, 2, one.n_meas()).astype(np.uint8)
    st1, pw1 = so.run(one, o1, [(list(one.inputs), vecs[1])],
                      mode=so.MODE_OWQS if mode == owqs.MODE_OWQS else so.MODE_EOWQS)
    p = owqs.Pattern(ctx, one)
    p.set_exec(owqs.EXEC_SUBSTATES)
    p.set_mode(mode)
    p.set_outcomes(o1)
    prof = p.run_profiled(cuda(vecs[1]))
    assert prof["tile(group)"]["launches"] > 0
    assert prof["tile(group)"]["bytes"] == prof["tile(group)"]["launches"] * 16 * 2 ** 16
    compare_factors(p, st1, one)
    if mode != owqs.MODE_EOWQS:
        np.testing.assert_allclose(p.read_probs(), pw1, atol=P_TOL)
    p.close()
