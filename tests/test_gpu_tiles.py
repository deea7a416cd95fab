"""GPU parity of the tile-fused passes (runs of windows / E / X / Z at live
widths >= 15 executed as one LDS-tiled pass each) against the FP64 oracle."""
import math

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
owqs = pytest.importorskip("paper_1604_05659_amd")

AMP_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return owqs.Context(0)


def _run(ctx, pattern, outcomes, inp, mode, exec_=owqs.EXEC_FUSED):
    p = owqs.Pattern(ctx, pattern)
    p.set_mode(mode)
    p.set_exec(exec_)
    p.set_outcomes(outcomes)
    x = None if inp is None else torch.as_tensor(inp).cuda()
    p.run(x)
    out = p.read_state().cpu().numpy().astype(np.complex128)
    probs = p.read_probs()
    info = p.plan_info()
    p.close()
    return out, probs, info


def random_windowed_pattern(g, n, n_ops):
    """n input qubits; a random mix of generalized windows (with E's to other
    live qubits and X/Z corrections on the new qubit), standalone E, X and Z
    steps with signals, and an occasional plain N ... M pair that breaks the
    tile groups."""
    live = list(range(n))
    nxt = n
    measured = []
    cmds = []
    for _ in range(n_ops):
        r = g.random()
        if r < 0.6:
            v = live[int(g.integers(len(live)))]
            w = nxt
            nxt += 1
            es = [("E", v, w)]
            others = [q for q in live if q != v]
            for x in g.choice(others, size=int(g.integers(0, 3)), replace=False):
                es.append(("E", v, int(x)))
            for y in g.choice(others, size=int(g.integers(0, 2)), replace=False):
                es.append(("E", w, int(y)))
            g.shuffle(es)
            s_dom = tuple(int(q) for q in g.choice(measured, size=min(len(measured), 1), replace=False)) \
                if measured and g.random() < 0.3 else ()
            cmds += [("N", w)] + [tuple(e) for e in es] + [("M", v, float(g.uniform(0, 2 * math.pi)), s_dom, ())]
            cmds.append(("X", w, (v,)))
            if g.random() < 0.5:
                cmds.append(("Z", w, (v,)))
            live[live.index(v)] = w
            measured.append(v)
        elif r < 0.8:
            a, b = g.choice(len(live), size=2, replace=False)
            cmds.append(("E", live[a], live[b]))
        elif r < 0.95 and measured:
            q = live[int(g.integers(len(live)))]
            cmds.append(("X" if g.random() < 0.5 else "Z", q, (measured[int(g.integers(len(measured)))],)))
        else:
            # an E between two other qubits inside the run keeps this from
            # being a window: plain N, E, E, M steps that end the tile group
            v = live[int(g.integers(len(live)))]
            u = nxt
            nxt += 1
            a, b = [q for q in live if q != v][:2]
            cmds += [("N", u), ("E", u, v), ("E", a, b), ("M", v, float(g.uniform(0, 2 * math.pi)), (), ())]
            live[live.index(v)] = u
            measured.append(v)
    return W.Pattern(list(range(n)), list(live), cmds)


@pytest.mark.parametrize("n", [15, 16, 18, 19, 21])
@pytest.mark.parametrize("mode", [owqs.MODE_OWQS, owqs.MODE_EOWQS_CHECK, owqs.MODE_EOWQS])
def test_random_windowed_patterns(ctx, n, mode, parity_report):
    g = np.random.default_rng(1800 + n)
    pat = random_windowed_pattern(g, n, 120)
    inp = W.gaussian_state(n, g)
    outc = g.integers(0, 2, size=pat.n_meas()).astype(np.uint8)
    want, pw = oc.run(pat, outc, inp.astype(np.complex128), oc.MODE_OWQS)
    if mode == owqs.MODE_OWQS:
        got, probs, info = _run(ctx, pat, outc, inp, mode)
        assert info[2] < info[1], info      # some runs were grouped
        err = float(np.max(np.abs(got - want)))
        parity_report(f"tiles_random_n{n}_owqs", max_amp_err=err, passes=info[2], steps=info[1])
        assert err <= AMP_TOL, err
        np.testing.assert_allclose(probs, pw, atol=1e-5)
    else:
        # random patterns have no flow: EOWQS keeps the fixed scale, so compare
        # directions (1 - F) and, in check mode, expect the determinism error
        p = owqs.Pattern(ctx, pat)
        p.set_mode(mode)
        p.set_exec(owqs.EXEC_FUSED)
        p.set_outcomes(outc)
        p.run(torch.as_tensor(inp).cuda())
        out = p.read_state(check=False).cpu().numpy().astype(np.complex128)
        f = abs(np.vdot(out, want)) ** 2 / (np.vdot(out, out).real * np.vdot(want, want).real)
        assert 1 - f <= 1e-8, 1 - f
        if mode == owqs.MODE_EOWQS_CHECK and np.max(np.abs(pw - 0.5)) > 1e-3:
            with pytest.raises(owqs.OwqsError) as e:
                p.check()
            assert e.value.status == owqs.E_NOT_DETERMINISTIC
        p.close()


@pytest.mark.parametrize("mode", [owqs.MODE_OWQS, owqs.MODE_EOWQS])
def test_flow_circuit_width_19(ctx, mode):
    wl = W.plain_large(n_logical=19, n_j=300, n_cz=60)
    want, pw = oc.run(wl.pattern, wl.outcomes, wl.input_state.astype(np.complex128),
                      oc.MODE_OWQS if mode == owqs.MODE_OWQS else oc.MODE_EOWQS)
    for ex in (owqs.EXEC_FUSED, owqs.EXEC_AUTO):
        got, probs, info = _run(ctx, wl.pattern, wl.outcomes, wl.input_state, mode, ex)
        assert info[2] * 4 < info[1]
        assert float(np.max(np.abs(got - want))) <= AMP_TOL
        if mode == owqs.MODE_OWQS:
            np.testing.assert_allclose(probs, pw, atol=1e-5)


def test_cluster_20_rows(ctx, parity_report):
    wl = W.cluster(rows=20, cols=10)
    want, pw = oc.run(wl.pattern, wl.outcomes)
    got, probs, info = _run(ctx, wl.pattern, wl.outcomes, None, owqs.MODE_OWQS)
    err = float(np.max(np.abs(got - want)))
    parity_report("cluster20x10_fused_tiles", max_amp_err=err, passes=info[2], steps=info[1])
    assert info[2] < info[1]
    assert err <= AMP_TOL
    np.testing.assert_allclose(probs, pw, atol=1e-5)


def test_autotuner_keeps_results(ctx):
    wl = W.plain_large(n_logical=20, n_j=200, n_cz=40)
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_outcomes(wl.outcomes)
    x = torch.as_tensor(wl.input_state).cuda()
    bits, ms = p.tune(x)
    assert 10 <= bits <= 13 and ms > 0
    p.run(x)
    got = p.read_state().cpu().numpy().astype(np.complex128)
    want, _ = oc.run(wl.pattern, wl.outcomes, wl.input_state.astype(np.complex128))
    assert float(np.max(np.abs(got - want))) <= AMP_TOL
    # a plan without tile passes has nothing to tune
    q = owqs.Pattern(ctx, W.plain_small().pattern)
    assert q.tune() == (0, 0.0)
    p.close()
    q.close()


def odd_even_window_pattern(g, n, n_win, even=True):
    """n input qubits; n_win windows N w; E's; M v; X w, each with E(v, w)
    once, twice (only if `even`) or three times, plus E's from v or w to
    other live qubits, and a standalone E now and then.  Returns the pattern
    and, per M, whether its E(v, w) count is odd."""
    live = list(range(n))
    nxt = n
    cmds, odd = [], []
    for _ in range(n_win):
        v = live[int(g.integers(len(live)))]
        w = nxt
        nxt += 1
        nvw = int(g.integers(1, 4)) if even else int(g.choice([1, 3]))
        others = [q for q in live if q != v]
        es = [("E", v, w)] * nvw
        es += [("E", v, int(x)) for x in g.choice(others, size=int(g.integers(0, 3)), replace=False)]
        es += [("E", w, int(y)) for y in g.choice(others, size=int(g.integers(0, 2)), replace=False)]
        es = [es[i] for i in g.permutation(len(es))]
        cmds += [("N", w)] + es + [("M", v, float(g.uniform(0, 2 * math.pi)), (), ()), ("X", w, (v,))]
        odd.append(nvw % 2 == 1)
        live[live.index(v)] = w
        if g.random() < 0.2:
            a, b = g.choice(len(live), size=2, replace=False)
            cmds.append(("E", live[a], live[b]))
    return W.Pattern(list(range(n)), live, cmds), np.array(odd)


@pytest.mark.parametrize("n,kind", [(10, "mixed"), (16, "mixed"), (16, "odd")])
@pytest.mark.parametrize("graph", [True, False])
def test_half_probability_windows(ctx, n, kind, graph):
    """OWQS mode: a window with an odd E(v, w) count has p = 1/2 exactly; run
    on its own (n = 10: one kernel per window) or in a tile pass whose
    windows are all such (kind "odd"), it records p = 1/2 without a
    reduction and leaves sigma to the next measurement that reduces.  Windows
    with an even count, and passes that hold one, reduce as before.  Against
    the oracle: the state and every probability, on two runs in a row."""
    g = np.random.default_rng(1900 + n + 7 * graph + (50 if kind == "odd" else 0))
    pat, odd = odd_even_window_pattern(g, n, 90, even=kind == "mixed")
    assert odd.any() and (kind == "odd" or not odd.all())
    inp = W.gaussian_state(n, g)
    for _ in range(20):   # forced outcomes of reasonable probability
        outc = g.integers(0, 2, size=pat.n_meas()).astype(np.uint8)
        want, pw = oc.run(pat, outc, inp.astype(np.complex128), oc.MODE_OWQS)
        if pw.min() > 1e-3:
            break
    assert pw.min() > 1e-3
    p = owqs.Pattern(ctx, pat)
    p.set_mode(owqs.MODE_OWQS)
    p.set_exec(owqs.EXEC_FUSED)
    p.set_graph(graph)
    p.set_outcomes(outc)
    x = torch.as_tensor(inp).cuda()
    for rep in range(2):   # the second run starts from the scale the first left
        p.run(x)
        got = p.read_state().cpu().numpy().astype(np.complex128)
        probs = p.read_probs()
        assert np.max(np.abs(got - want)) <= AMP_TOL, rep
        np.testing.assert_allclose(probs, pw, atol=1e-5)
        if n < 15 or kind == "odd":
            assert np.all(probs[odd] == 0.5)
    prof = p.run_profiled(x)
    if n >= 15:
        assert p.plan_info()[2] < p.plan_info()[1]
        assert prof["tile(group)"]["launches"] > 0
    if kind == "odd":   # no reduction anywhere: no finishing kernel
        assert prof.get("finish(FP64)", {"launches": 0})["launches"] == 0
    got = p.read_state().cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - want)) <= AMP_TOL
    p.close()


@pytest.mark.parametrize("graph", [True, False])
def test_half_windows_renormalise_long_runs(ctx, graph):
    """OWQS mode, 600 windows that all have p = 1/2 exactly (odd E(v, w)
    counts) at width 16: far more than may pass without a renormalisation,
    so tile passes of them now and then sum the norm of their output alone
    and reset sigma from it (one finishing kernel each, no window sums).
    Every probability is exactly 1/2 and the state matches the oracle, on
    the fused executor, on two runs in a row, in a batched run of two
    inputs (the multi-pattern tile and finishing kernels), and in the
    allocation-free run."""
    g = np.random.default_rng(2401 + graph)
    pat, odd = odd_even_window_pattern(g, 16, 600, even=False)
    assert odd.all()
    outc = g.integers(0, 2, size=pat.n_meas()).astype(np.uint8)
    inps = [W.gaussian_state(16, g) for _ in range(2)]
    wants = [oc.run(pat, outc, x.astype(np.complex128), oc.MODE_OWQS) for x in inps]
    for want, pw in wants:   # 1/2 up to the rounding of the complex64 input
        np.testing.assert_allclose(pw, 0.5, rtol=0, atol=1e-8)
    p = owqs.Pattern(ctx, pat)
    p.set_mode(owqs.MODE_OWQS)
    p.set_exec(owqs.EXEC_FUSED)
    p.set_graph(graph)
    p.set_outcomes(outc)
    x = torch.as_tensor(inps[0]).cuda()
    for rep in range(2):
        p.run(x)
        got = p.read_state().cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(got - wants[0][0])) <= AMP_TOL, rep
        assert np.all(p.read_probs() == 0.5), rep
    prof = p.run_profiled(x)
    width, nsteps, npasses = p.plan_info()
    assert width == 16 and npasses < nsteps
    assert prof["tile(group)"]["launches"] >= 600 // 64
    # renormalisations happen, far fewer than the passes
    fin = prof.get("finish(FP64)", {"launches": 0})["launches"]
    assert 0 < fin < prof["tile(group)"]["launches"]
    got = p.read_state().cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - wants[0][0])) <= AMP_TOL
    # a batched run: both inputs through the multi-pattern kernels
    q = owqs.Pattern(ctx, pat)
    q.set_mode(owqs.MODE_OWQS)
    q.set_exec(owqs.EXEC_FUSED)
    q.set_outcomes(outc)
    ins = [torch.as_tensor(v).cuda() for v in inps]
    outs = [torch.empty(1 << 16, dtype=torch.complex64, device="cuda") for _ in inps]
    owqs.run_batch(ctx, [p, q], ins, outs)
    torch.cuda.synchronize()
    for o, (want, _) in zip(outs, wants):
        assert np.max(np.abs(o.cpu().numpy().astype(np.complex128) - want)) <= AMP_TOL
    # the allocation-free run of the same plan (uploaded by the runs above)
    p.run(x)
    out = torch.empty(1 << 16, dtype=torch.complex64, device="cuda")
    probs = torch.empty(pat.n_meas(), dtype=torch.float64, device="cuda")
    p.run_noalloc(x, out, probs)
    torch.cuda.synchronize()
    assert np.max(np.abs(out.cpu().numpy().astype(np.complex128) - wants[0][0])) <= AMP_TOL
    assert np.all(probs.cpu().numpy() == 0.5)
    p.close()
    q.close()


@pytest.mark.parametrize("n,exec_", [(10, owqs.EXEC_AUTO), (10, owqs.EXEC_FUSED), (16, owqs.EXEC_FUSED),
                                     (16, owqs.EXEC_SUBSTATES)])
def test_sum_all_sums_every_window(ctx, n, exec_):
    """owqs_set_sum_all(1): windows with p = 1/2 exactly are summed like every
    other M (no 1/2 recorded without a sum, every pass with windows has a
    finishing reduction); the state and every probability still match the
    oracle, and switching back restores the default plan."""
    g = np.random.default_rng(2600 + n + exec_)
    pat, odd = odd_even_window_pattern(g, n, 90, even=False)
    inp = W.gaussian_state(n, g)
    outc = g.integers(0, 2, size=pat.n_meas()).astype(np.uint8)
    want, pw = oc.run(pat, outc, inp.astype(np.complex128), oc.MODE_OWQS)
    p = owqs.Pattern(ctx, pat)
    p.set_mode(owqs.MODE_OWQS)
    p.set_exec(exec_)
    p.set_outcomes(outc)
    x = torch.as_tensor(inp).cuda()
    p.set_sum_all(True)
    p.run(x)
    got = p.read_state().cpu().numpy().astype(np.complex128)
    probs = p.read_probs()
    assert np.max(np.abs(got - want)) <= AMP_TOL
    np.testing.assert_allclose(probs, pw, atol=1e-5)
    assert np.all(odd) and not np.any(probs == 0.5), "every window summed"
    if exec_ == owqs.EXEC_FUSED:
        prof = p.run_profiled(x)
        assert prof.get("finish(FP64)", {"launches": 0})["launches"] > 0
    p.set_sum_all(False)
    p.run(x)
    got = p.read_state().cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - want)) <= AMP_TOL
    if exec_ != owqs.EXEC_SUBSTATES:
        assert np.all(p.read_probs() == 0.5)
    p.close()


def runs_circuit(g, n, n_gates, hot=3, p_cz=0.08):
    """J gates mostly on a few wires (long runs of windows on one slot, which
    the plan composes into 2x2 maps), CZ now and then on random pairs."""
    gates = []
    for _ in range(n_gates):
        if g.random() < p_cz:
            a, b = g.choice(n, size=2, replace=False)
            gates.append(("CZ", int(a), int(b)))
        else:
            q = int(g.integers(hot)) if g.random() < 0.7 else int(g.integers(n))
            gates.append(("J", q, float(g.uniform(0, 2 * math.pi))))
    return gates


@pytest.mark.parametrize("n,bits", [(16, 10), (18, 12), (20, 11)])
@pytest.mark.parametrize("mode", [owqs.MODE_OWQS, owqs.MODE_EOWQS])
def test_composed_window_runs(ctx, n, bits, mode, parity_report):
    """Runs of windows on one round position composed into one 2x2 map
    (products of the windows' maps, pending signs taken into the map; every
    round window of a pass becomes a map, runs of one included):
    state and probabilities against the oracle, on two runs in a row, and
    the same state with every window summed (no composition)."""
    g = np.random.default_rng(2300 + n + 5 * mode)
    gates = runs_circuit(g, n, 260)
    pat = W.circuit_to_pattern(n, gates)
    inp = W.gaussian_state(n, g)
    outc = g.integers(0, 2, size=pat.n_meas()).astype(np.uint8)
    want, pw = oc.run(pat, outc, inp.astype(np.complex128),
                      oc.MODE_OWQS if mode == owqs.MODE_OWQS else oc.MODE_EOWQS)
    p = owqs.Pattern(ctx, pat)
    p.set_mode(mode)
    p.set_exec(owqs.EXEC_FUSED)
    p.set_outcomes(outc)
    p.set_tile_bits(bits)
    alone, maps, inside = p.plan_tile_work()
    assert maps > 0 and inside > maps, (alone, maps, inside)
    x = torch.as_tensor(inp).cuda()
    for rep in range(2):
        p.run(x)
        got = p.read_state().cpu().numpy().astype(np.complex128)
        err = float(np.max(np.abs(got - want)))
        assert err <= AMP_TOL, (rep, err)
        if mode == owqs.MODE_OWQS:
            np.testing.assert_allclose(p.read_probs(), pw, atol=1e-5)
    parity_report(f"composed_runs_n{n}_k{bits}_mode{mode}", max_amp_err=err, maps=maps, windows_in_maps=inside)
    if mode == owqs.MODE_OWQS:
        p.set_sum_all(True)
        assert p.plan_tile_work()[1] == 0
        p.run(x)
        got2 = p.read_state().cpu().numpy().astype(np.complex128)
        assert float(np.max(np.abs(got2 - want))) <= AMP_TOL
    p.close()
