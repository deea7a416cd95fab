"""GPU parity of drawn outcomes (Fig. 6 sampling on the device) against the
FP64 oracle's sampled runs with the same uniforms.

Both sides decide o = 0 when u <= p_0; the GPU's p_0 comes from complex64
amplitudes (FP64 sums), the oracle's from complex128, so they differ by
~1e-7.  Uniforms are therefore drawn at least 1e-4 away from every p_0 of the
oracle's run (re-drawn otherwise, seeded); then the outcome strings must be
identical and the amplitudes within 1e-5."""
import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
owqs = pytest.importorskip("paper_1604_05659_amd")

AMP_TOL = 1e-5
MARGIN = 1e-4


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return owqs.Context(0)


def safe_uniforms(pat, inp, g, tries=50):
    """Uniforms with every oracle p_0 at least MARGIN away; returns them with
    the oracle's (psi, probs, outcomes)."""
    ref_in = None if inp is None else inp.astype(np.complex128)
    for _ in range(tries):
        u = g.random(pat.n_meas())
        psi, probs, outc = oc.run_sampled(pat, u, ref_in)
        p0 = np.where(outc == 0, probs, 1.0 - probs)
        if pat.n_meas() == 0 or np.min(np.abs(u - p0)) >= MARGIN:
            return u, psi, probs, outc
    pytest.skip("no uniforms away from the decision boundaries")


def run_gpu(ctx, pat, u, inp, graph=True):
    p = owqs.Pattern(ctx, pat)
    p.set_graph(graph)
    p.set_uniforms(u)
    p.run(None if inp is None else torch.as_tensor(inp).cuda())
    out = p.read_state().cpu().numpy().astype(np.complex128)
    return p, out, p.read_probs(), p.read_outcomes()


def test_random_patterns(ctx, parity_report):
    g = np.random.default_rng(606)
    worst = 0.0
    for _ in range(30):
        pat = W.random_pattern(g, max_qubits=10)
        inp = W.gaussian_state(len(pat.inputs), g) if pat.inputs else None
        u, want, pw, ow = safe_uniforms(pat, inp, g)
        p, got, probs, outc = run_gpu(ctx, pat, u, inp)
        np.testing.assert_array_equal(outc, ow)
        err = float(np.max(np.abs(got - want))) if got.size else 0.0
        worst = max(worst, err)
        assert err <= AMP_TOL
        np.testing.assert_allclose(probs, pw, atol=1e-5)
        p.close()
    parity_report("sampled_random_patterns", max_amp_err=worst)


@pytest.mark.parametrize("graph", [True, False])
def test_circuit_width_17_repeated_draws(ctx, graph, parity_report):
    """A J/CZ circuit pattern at live width 16 <-> 17 (probability passes over
    several grid blocks), drawn three times with new uniforms on one pattern
    (graph replays with the uniforms re-uploaded)."""
    wl = W.plain_large(n_logical=16, n_j=120, n_cz=24)
    g = np.random.default_rng(17)
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_graph(graph)
    x = torch.as_tensor(wl.input_state).cuda()
    for rep in range(3):
        u, want, pw, ow = safe_uniforms(wl.pattern, wl.input_state, g)
        p.set_uniforms(u)
        p.run(x)
        got = p.read_state().cpu().numpy().astype(np.complex128)
        np.testing.assert_array_equal(p.read_outcomes(), ow)
        err = float(np.max(np.abs(got - want)))
        assert err <= AMP_TOL, (rep, err)
        np.testing.assert_allclose(p.read_probs(), pw, atol=1e-5)
        # a J/CZ pattern with its corrections is deterministic: p = 1/2 and
        # the output does not depend on what was drawn
        np.testing.assert_allclose(p.read_probs(), 0.5, atol=1e-5)
    parity_report(f"sampled_width17_graph{int(graph)}", max_amp_err=err)
    # back to forced outcomes
    p.set_outcomes(wl.outcomes)
    p.run(x)
    forced = p.read_state().cpu().numpy().astype(np.complex128)
    np.testing.assert_array_equal(p.read_outcomes(), wl.outcomes)
    assert float(np.max(np.abs(forced - got))) <= 1e-4
    p.close()


def test_sampling_state_rules(ctx):
    wl = W.plain_small()
    p = owqs.Pattern(ctx, wl.pattern)
    u = np.full(p.n_meas, 0.5)
    p.set_mode(owqs.MODE_EOWQS)
    p.set_uniforms(u)
    with pytest.raises(owqs.OwqsError) as e:
        p.run(None)
    assert e.value.status == owqs.E_STATE
    p.set_mode(owqs.MODE_OWQS)
    p.run(None)
    out = torch.empty(16, dtype=torch.complex64, device="cuda")
    with pytest.raises(owqs.OwqsError) as e:
        owqs.run_batch(ctx, [p], [None], [out])
    assert e.value.status == owqs.E_STATE
    with pytest.raises(owqs.OwqsError):
        p.set_uniforms(np.full(p.n_meas, 1.0))
    p.set_uniforms(None)
    owqs.run_batch(ctx, [p], [None], [out])
    p.close()


@pytest.mark.parametrize("nl,nj,ncz", [(6, 60, 12), (17, 80, 16)])
def test_drawn_windows_on_the_fused_plan(ctx, nl, nj, ncz):
    """Every M of a J/CZ circuit is a window with p = 1/2, so with the fused
    executors one device kernel resolves every outcome, coefficient and
    folded correction from the uniforms and the fused plan (tile passes at
    width 17) runs with those tables, all in one graph; the plain executor
    draws window by window on the device.  Both give the oracle's outcome
    string and output, on two draws in a row."""
    g = np.random.default_rng(nl)
    pat = W.circuit_to_pattern(nl, W.random_jcz_circuit(nl, nj, ncz, g))
    inp = W.gaussian_state(nl, g)
    for draw in range(2):
        u, want, pw, ow = safe_uniforms(pat, inp, g)
        for ex in (owqs.EXEC_AUTO, owqs.EXEC_FUSED, owqs.EXEC_PLAIN):
            p = owqs.Pattern(ctx, pat)
            p.set_exec(ex)
            p.set_uniforms(u)
            for rep in range(2):  # the second run replays the captured graph
                p.run(torch.as_tensor(inp).cuda())
                got = p.read_state().cpu().numpy().astype(np.complex128)
                assert np.array_equal(p.read_outcomes(), ow), (draw, ex, rep)
                assert np.max(np.abs(got - want)) <= AMP_TOL, (draw, ex, rep)
                np.testing.assert_allclose(p.read_probs(), pw, atol=1e-5)
            p.close()


@pytest.mark.parametrize("exec_", [owqs.EXEC_PLAIN, owqs.EXEC_FUSED])
def test_long_runs_of_drawn_windows(ctx, exec_):
    """300 drawn windows (p = 1/2 exactly) in a row, more than the 128 that
    may skip their sum before one renormalises: outcomes, output, norm and
    probabilities against the oracle, for the device-drawn plain plan and
    the fused plan."""
    wl = W.plain_large(index=5, n_logical=10, n_j=300, n_cz=30)
    g = np.random.default_rng(300)
    u, want, pw, ow = safe_uniforms(wl.pattern, wl.input_state, g)
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_exec(exec_)
    p.set_uniforms(u)
    p.run(torch.as_tensor(wl.input_state).cuda())
    got = p.read_state().cpu().numpy().astype(np.complex128)
    np.testing.assert_array_equal(p.read_outcomes(), ow)
    assert float(np.max(np.abs(got - want))) <= AMP_TOL
    assert abs(np.linalg.norm(got) - 1) <= 1e-5
    np.testing.assert_allclose(p.read_probs(), pw, atol=1e-5)
    p.close()


def test_fused_drawn_plan_replays_with_new_uniforms(ctx, parity_report):
    """The fused drawn plan (tile passes at width 18) is captured once and
    replayed with a new set of uniforms before every run, with unrelated
    eager work in between; every replay gives the oracle's outcomes,
    output and probabilities for its uniforms."""
    g = np.random.default_rng(1818)
    nl = 18
    pat = W.circuit_to_pattern(nl, W.random_jcz_circuit(nl, 90, 14, g))
    inp = W.gaussian_state(nl, g)
    x = torch.as_tensor(inp).cuda()
    p = owqs.Pattern(ctx, pat)
    p.set_exec(owqs.EXEC_FUSED)
    worst = 0.0
    for draw in range(4):
        u, want, pw, ow = safe_uniforms(pat, inp, g)
        p.set_uniforms(u)
        junk = torch.randn(1 << 18, device="cuda").cumsum(0)   # unrelated eager work
        p.run(x)
        got = p.read_state().cpu().numpy().astype(np.complex128)
        assert np.array_equal(p.read_outcomes(), ow), draw
        err = float(np.max(np.abs(got - want)))
        worst = max(worst, err)
        assert err <= AMP_TOL, (draw, err)
        np.testing.assert_allclose(p.read_probs(), pw, atol=1e-5)
        del junk
    parity_report("drawn_fused_replays_width18", max_amp_err=worst)
    p.close()
