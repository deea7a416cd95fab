"""GPU parity of the batched forms: LDS-resident runs over basis inputs
(recognition problem), over arbitrary input states, heterogeneous pattern
batches, and the HIP-graph replay of a plan."""
import math

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc
from oracle import reference as ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
owqs = pytest.importorskip("paper_1604_05659_amd")

AMP_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return owqs.Context(0)


def _load(ctx, pattern, outcomes, mode=owqs.MODE_OWQS, exec_=owqs.EXEC_FUSED):
    p = owqs.Pattern(ctx, pattern)
    p.set_mode(mode)
    p.set_exec(exec_)
    p.set_outcomes(outcomes)
    return p


@pytest.mark.parametrize("mode", [owqs.MODE_OWQS, owqs.MODE_EOWQS])
@pytest.mark.parametrize("exec_", [owqs.EXEC_PLAIN, owqs.EXEC_FUSED])
def test_basis_columns_small(ctx, mode, exec_):
    wl = W.recognition(n_logical=5, n_j=40, n_cz=8)
    u = ref.circuit_unitary(5, wl.meta["gates"])
    p = _load(ctx, wl.pattern, wl.outcomes, mode, exec_)
    probs = torch.zeros((32, p.n_meas), dtype=torch.float64, device="cuda")
    out = p.run_basis(0, 32, probs=probs)
    p.check()
    got = out.cpu().numpy().astype(np.complex128)
    np.testing.assert_allclose(got.T, u, atol=AMP_TOL)
    if mode == owqs.MODE_OWQS:
        np.testing.assert_allclose(probs.cpu().numpy(), 0.5, atol=1e-5)
    # a sub-range gives the same columns
    part = p.run_basis(7, 9).cpu().numpy().astype(np.complex128)
    np.testing.assert_allclose(part, got[7:16], atol=0)
    p.close()


def test_recognition_full_size(ctx, parity_report):
    """12 inputs, 300 J + 60 CZ, all 4096 basis inputs: columns sampled against
    the oracle, and the whole matrix checked for unitarity."""
    wl = W.recognition()
    p = _load(ctx, wl.pattern, wl.outcomes, owqs.MODE_EOWQS)
    assert p.plan_info()[0] <= 14
    out = p.run_basis()
    p.check()
    torch.cuda.synchronize()
    g = np.random.default_rng(4096)
    cols = sorted(set([0, 1, 4095] + list(g.choice(4096, 13, replace=False))))
    worst = 0.0
    for k in cols:
        want, _ = oc.run(wl.pattern, wl.outcomes, W.basis_state(12, k).astype(np.complex128), oc.MODE_EOWQS)
        got = out[k].cpu().numpy().astype(np.complex128)
        worst = max(worst, float(np.max(np.abs(got - want))))
    uh = out.transpose(0, 1).contiguous()            # U with columns = outputs
    gram = torch.matmul(uh.conj().transpose(0, 1).contiguous(), uh)
    eye = torch.eye(4096, dtype=torch.complex64, device="cuda")
    unit_err = float((gram - eye).abs().max().item())
    parity_report("recognition_4096_columns", max_amp_err_sampled=worst, max_unitarity_err=unit_err,
                  columns_checked=len(cols))
    assert worst <= AMP_TOL
    assert unit_err <= 1e-4
    p.close()


def test_run_states_matches_oracle(ctx):
    wl = W.plain_large(n_logical=9, n_j=120, n_cz=20)
    p = _load(ctx, wl.pattern, wl.outcomes)
    g = np.random.default_rng(3)
    states = np.stack([W.gaussian_state(9, g) for _ in range(24)])
    out = p.run_states(torch.as_tensor(states).cuda())
    p.check()
    got = out.cpu().numpy().astype(np.complex128)
    for k in range(24):
        want, _ = oc.run(wl.pattern, wl.outcomes, states[k].astype(np.complex128))
        np.testing.assert_allclose(got[k], want, atol=AMP_TOL)
    p.close()


def test_run_states_long_runs_of_half_windows(ctx):
    """OWQS, LDS-resident: 300 windows with p = 1/2 (odd E(v, w) count) are
    recorded without the block sum, at most 128 in a row before one sums
    and renormalises; states, norms and probabilities against the oracle."""
    wl = W.plain_large(index=3, n_logical=8, n_j=300, n_cz=40)
    p = _load(ctx, wl.pattern, wl.outcomes)
    assert p.plan_info()[0] <= 14
    g = np.random.default_rng(31)
    states = np.stack([W.gaussian_state(8, g) for _ in range(6)])
    probs = torch.zeros((6, p.n_meas), dtype=torch.float64, device="cuda")
    out = p.run_states(torch.as_tensor(states).cuda(), probs=probs)
    p.check()
    got = out.cpu().numpy().astype(np.complex128)
    pr = probs.cpu().numpy()
    for k in range(6):
        want, pw = oc.run(wl.pattern, wl.outcomes, states[k].astype(np.complex128))
        np.testing.assert_allclose(got[k], want, atol=AMP_TOL)
        assert abs(np.linalg.norm(got[k]) - 1) <= 1e-5
        np.testing.assert_allclose(pr[k], pw, atol=1e-5)
    p.close()


def test_heterogeneous_batch(ctx, parity_report):
    """Batch of patterns with uneven widths (LDS-resident and wide ones),
    against the oracle one by one."""
    wls = [W.batched_random(i, w_lo=6, w_hi=18, c_lo=30, c_hi=300) for i in range(40)]
    pats, ins, outs = [], [], []
    for wl in wls:
        p = _load(ctx, wl.pattern, wl.outcomes)
        pats.append(p)
        ins.append(torch.as_tensor(wl.input_state).cuda())
        outs.append(torch.empty(1 << len(wl.pattern.outputs), dtype=torch.complex64, device="cuda"))
    widths = [p.plan_info()[0] for p in pats]
    assert min(widths) <= 14 < max(widths)
    for rep in range(2):
        owqs.run_batch(ctx, pats, ins, outs)
        torch.cuda.synchronize()
        worst = 0.0
        for wl, p, o in zip(wls, pats, outs):
            p.check()
            want, pw = oc.run(wl.pattern, wl.outcomes, wl.input_state.astype(np.complex128))
            got = o.cpu().numpy().astype(np.complex128)
            worst = max(worst, float(np.max(np.abs(got - want))))
            np.testing.assert_allclose(p.read_probs(), pw, atol=1e-5)
        parity_report(f"batched_random_40_rep{rep}", max_amp_err=worst)
        assert worst <= AMP_TOL
    for p in pats:
        p.close()


def test_batch_reports_zero_probability_per_pattern(ctx):
    good = W.plain_small()
    bad = W.Pattern([], [1], [("N", 0), ("N", 1), ("M", 0, 0.0, (), ())])
    pg = _load(ctx, good.pattern, good.outcomes)
    pb = _load(ctx, bad, [1])
    og = torch.empty(16, dtype=torch.complex64, device="cuda")
    ob = torch.empty(2, dtype=torch.complex64, device="cuda")
    owqs.run_batch(ctx, [pg, pb], [None, None], [og, ob])
    pg.check()
    with pytest.raises(owqs.OwqsError) as e:
        pb.check()
    assert e.value.status == owqs.E_ZERO_PROB
    want, _ = oc.run(good.pattern, good.outcomes)
    np.testing.assert_allclose(og.cpu().numpy(), want, atol=AMP_TOL)
    pg.close()
    pb.close()


def test_graph_replay_matches_eager(ctx):
    """The captured plan replayed several times, with eager work and
    synchronisations in between, gives the eager result every time."""
    wl = W.plain_large(n_logical=14, n_j=150, n_cz=25)
    inp = torch.as_tensor(wl.input_state).cuda()
    for exec_ in (owqs.EXEC_PLAIN, owqs.EXEC_FUSED):
        p = _load(ctx, wl.pattern, wl.outcomes, owqs.MODE_OWQS, exec_)
        p.set_graph(False)
        p.run(inp)
        eager = p.read_state().clone()
        p.set_graph(True)
        for rep in range(4):
            junk = torch.randn(1 << 16, device="cuda").sum()      # unrelated eager work
            p.run(inp)
            got = p.read_state()
            torch.cuda.synchronize()
            assert float((got - eager).abs().max().item()) == 0.0, rep
            del junk
        # new outcomes invalidate and recapture the graph
        other = W.outcome_bits(wl.pattern.n_meas(), np.random.default_rng(9))
        p.set_outcomes(other)
        p.run(inp)
        got = p.read_state().cpu().numpy().astype(np.complex128)
        want, _ = oc.run(wl.pattern, other, wl.input_state.astype(np.complex128))
        np.testing.assert_allclose(got, want, atol=AMP_TOL)
        p.close()


def test_tune_batch_keeps_results(ctx):
    """owqs_tune_batch times the batch at every tile size and keeps the
    fastest on the wide patterns; the batch then still gives the oracle's
    outputs and probabilities."""
    wls = [W.batched_random(i, w_lo=12, w_hi=19, c_lo=40, c_hi=200) for i in range(24)]
    pats, ins, outs = [], [], []
    for wl in wls:
        p = _load(ctx, wl.pattern, wl.outcomes)
        pats.append(p)
        ins.append(torch.as_tensor(wl.input_state).cuda())
        outs.append(torch.empty(1 << len(wl.pattern.outputs), dtype=torch.complex64, device="cuda"))
    assert max(p.plan_info()[0] for p in pats) > 14
    bits, ms = owqs.tune_batch(ctx, pats, ins, outs)
    assert 10 <= bits <= 13 and ms > 0.0
    owqs.run_batch(ctx, pats, ins, outs)
    torch.cuda.synchronize()
    for wl, p, o in zip(wls, pats, outs):
        p.check()
        want, pw = oc.run(wl.pattern, wl.outcomes, wl.input_state.astype(np.complex128))
        np.testing.assert_allclose(o.cpu().numpy().astype(np.complex128), want, atol=AMP_TOL)
        np.testing.assert_allclose(p.read_probs(), pw, atol=1e-5)
    for p in pats:
        p.close()
