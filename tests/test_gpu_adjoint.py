"""GPU parity of the adjoint gradient d(sum_i <Z_i>)/d(alpha) against the FP64
oracle's exact parameter-shift gradient (and central differences), plus
properties that hold at full size: checkpoint strides agree, the GPU's own
shift rule agrees with its adjoint, and the torch.autograd wrapper returns
the same gradient.

Tolerance for gradients: |dg| <= 1e-4 * max(1, |g|); losses within 1e-5.
"""
import math

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
owqs = pytest.importorskip("paper_1604_05659_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return owqs.Context(0)


def _gtol(g):
    return 1e-4 * np.maximum(1.0, np.abs(g))


def _load(ctx, wl):
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_EOWQS)
    p.set_outcomes(wl.outcomes)
    return p


def test_adjoint_small_against_oracle(ctx, parity_report):
    wl, sets = W.ansatz(n_logical=4, layers=3, batch=4)
    p = _load(ctx, wl)
    loss, grad = p.adjoint(sets)
    loss, grad = loss.cpu().numpy(), grad.cpu().numpy()
    worst = 0.0
    for b in range(4):
        want_l = oc.loss_at(wl.pattern, wl.outcomes, sets[b])
        assert abs(loss[b] - want_l) <= 1e-5
        g_shift = oc.param_shift_grad(wl.pattern, wl.outcomes, sets[b])
        g_fd = oc.central_fd_grad(wl.pattern, wl.outcomes, sets[b], h=1e-4)
        assert np.all(np.abs(grad[b] - g_shift) <= _gtol(g_shift)), np.max(np.abs(grad[b] - g_shift))
        assert np.all(np.abs(grad[b] - g_fd) <= _gtol(g_fd))
        worst = max(worst, float(np.max(np.abs(grad[b] - g_shift))))
    parity_report("adjoint_ansatz4x3", max_abs_grad_err=worst)
    p.close()


def test_adjoint_with_inputs_and_observable_subset(ctx):
    wl = W.plain_large(n_logical=6, n_j=40, n_cz=8)
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_EOWQS)
    p.set_outcomes(wl.outcomes)
    g = np.random.default_rng(11)
    base = wl.pattern.angles()
    sets = np.stack([base, base + g.normal(0, 0.3, base.size)])
    x = torch.as_tensor(wl.input_state).cuda()
    obs = [0, 2, 5]
    loss, grad = p.adjoint(sets, obs, x)
    inp = wl.input_state.astype(np.complex128)
    for b in range(2):
        want_l = oc.loss_at(wl.pattern, wl.outcomes, sets[b], inp, obs=obs)
        assert abs(loss[b].item() - want_l) <= 1e-5
        g_shift = oc.param_shift_grad(wl.pattern, wl.outcomes, sets[b], inp, obs=obs)
        gg = grad[b].cpu().numpy()
        assert np.all(np.abs(gg - g_shift) <= _gtol(g_shift)), np.max(np.abs(gg - g_shift))
    p.close()


def test_checkpoint_strides_agree(ctx):
    """The recomputing sweep (negative strides) gives bit-identical results for
    every segment length; the reversing sweep (grouped forward, windows
    inverted backward, each segment restarted from its checkpoint) agrees
    with it to FP32 rounding: losses within 1e-6, gradients within 1e-5."""
    wl, sets = W.ansatz(n_logical=6, layers=5, batch=3)
    p = _load(ctx, wl)
    ref = None
    for stride in (-1, -3, -6, -16, -1000):
        loss, grad = p.adjoint(sets, ckpt_stride=stride)
        torch.cuda.synchronize()
        if ref is None:
            ref = (loss.clone(), grad.clone())
        else:
            assert torch.equal(loss, ref[0]) and torch.equal(grad, ref[1]), stride
    for stride in (1, 3, 6, 16, 1000):
        loss, grad = p.adjoint(sets, ckpt_stride=stride)
        torch.cuda.synchronize()
        # the forward sweep runs grouped (tile passes) here, per step there
        assert float((loss - ref[0]).abs().max()) <= 1e-6, stride
        d = (grad - ref[1]).abs()
        assert bool((d <= 1e-5 * torch.clamp(ref[1].abs(), min=1.0)).all()), (stride, float(d.max()))
    p.close()


def test_reversing_sweep_matches_recompute_at_full_size(ctx, parity_report):
    """16 qubits, 25 layers, 64 sets: the two backward sweeps agree."""
    wl, sets = W.ansatz()
    p = _load(ctx, wl)
    l_rev, g_rev = p.adjoint(sets)
    l_rev, g_rev = l_rev.clone(), g_rev.clone()
    l_rec, g_rec = p.adjoint(sets, ckpt_stride=-16)
    assert float((l_rev - l_rec).abs().max()) <= 1e-6
    d = float((g_rev - g_rec).abs().max())
    parity_report("adjoint_reverse_vs_recompute_16x25", max_abs_grad_diff=d)
    assert d <= 1e-5, d
    p.close()


def test_full_size_gradient(ctx, parity_report):
    """16 qubits, 25 layers, 400 angles, 64 angle sets."""
    wl, sets = W.ansatz()
    p = _load(ctx, wl)
    loss, grad = p.adjoint(sets)
    loss, grad = loss.cpu().numpy(), grad.cpu().numpy()
    assert grad.shape == (64, 400)
    rng = np.random.default_rng(400)
    # oracle: losses of two sets, exact shift-rule gradient at sampled entries
    worst_l, worst_g = 0.0, 0.0
    for b in (0, 37):
        want = oc.loss_at(wl.pattern, wl.outcomes, sets[b])
        worst_l = max(worst_l, abs(loss[b] - want))
        idx = sorted(rng.choice(400, 5, replace=False).tolist() + [0, 399])
        g_shift = oc.param_shift_grad(wl.pattern, wl.outcomes, sets[b], indices=idx)
        d = np.abs(grad[b, idx] - g_shift[idx])
        assert np.all(d <= _gtol(g_shift[idx])), d
        worst_g = max(worst_g, float(d.max()))
    assert worst_l <= 1e-5
    # the GPU's own shift rule at sampled (set, angle) pairs, all in one batch
    picks = [(int(rng.integers(64)), int(rng.integers(400))) for _ in range(16)]
    shifted = []
    for b, k in picks:
        for sgn in (1, -1):
            a = sets[b].copy()
            a[k] += sgn * math.pi / 2
            shifted.append(a)
    sl, _ = p.adjoint(np.stack(shifted))
    sl = sl.cpu().numpy()
    worst_s = 0.0
    for i, (b, k) in enumerate(picks):
        gs = 0.5 * (sl[2 * i] - sl[2 * i + 1])
        worst_s = max(worst_s, abs(gs - grad[b, k]))
        assert abs(gs - grad[b, k]) <= 1e-4 * max(1.0, abs(gs))
    parity_report("adjoint_ansatz16x25_batch64", max_abs_loss_err=worst_l, max_abs_grad_err_vs_oracle=worst_g,
                  max_abs_grad_err_vs_gpu_shift=worst_s)
    p.close()


def test_autograd_function(ctx):
    wl, sets = W.ansatz(n_logical=5, layers=4, batch=3)
    p = _load(ctx, wl)
    alphas = torch.tensor(sets, dtype=torch.float64, requires_grad=True)
    loss = owqs.pattern_loss(p, alphas)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64)
    (loss * w).sum().backward()
    ref_l, ref_g = p.adjoint(sets)
    np.testing.assert_allclose(loss.detach().numpy(), ref_l.cpu().numpy(), atol=0)
    np.testing.assert_allclose(alphas.grad.numpy(), (w[:, None] * ref_g.cpu()).numpy(), rtol=1e-12, atol=1e-15)
    p.close()


def test_adjoint_rejects_measurements_outside_windows(ctx):
    wl = W.cluster(rows=3, cols=4)
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_outcomes(wl.outcomes)
    with pytest.raises(owqs.OwqsError) as e:
        p.adjoint(np.zeros((1, p.n_meas)))
    assert e.value.status == owqs.E_STATE
    p.close()


def _masked_window_pattern(g, n, n_ops):
    """n inputs; windows whose runs also hold E's from v or w to other live
    qubits (sign masks), standalone E and signalled X/Z steps: no measurement
    outside a window, as the adjoint requires.  No flow, but every window is
    invertible (one E between v and w)."""
    live = list(range(n))
    nxt, measured, cmds = n, [], []
    for _ in range(n_ops):
        r = g.random()
        if r < 0.7:
            v = live[int(g.integers(len(live)))]
            w = nxt
            nxt += 1
            others = [q for q in live if q != v]
            es = [("E", v, w)]
            es += [("E", v, int(x)) for x in g.choice(others, size=int(g.integers(0, 3)), replace=False)]
            es += [("E", w, int(y)) for y in g.choice(others, size=int(g.integers(0, 2)), replace=False)]
            g.shuffle(es)
            cmds += [("N", w)] + [tuple(e) for e in es] + [("M", v, float(g.uniform(0, 2 * math.pi)), (), ())]
            cmds.append(("X", w, (v,)))
            live[live.index(v)] = w
            measured.append(v)
        elif r < 0.85:
            a, b = g.choice(len(live), size=2, replace=False)
            cmds.append(("E", live[a], live[b]))
        elif measured:
            q = live[int(g.integers(len(live)))]
            cmds.append(("X" if g.random() < 0.5 else "Z", q, (measured[int(g.integers(len(measured)))],)))
    return W.Pattern(list(range(n)), list(live), cmds)


def test_masked_windows_reversing_tiled_sweep(ctx, parity_report):
    """Width 16 (tile passes), windows with sign masks: the reversing sweep
    agrees with the recomputing per-step sweep, and with the shift rule
    evaluated on GPU forward losses."""
    g = np.random.default_rng(1616)
    pat = _masked_window_pattern(g, 16, 160)
    p = owqs.Pattern(ctx, pat)
    p.set_mode(owqs.MODE_EOWQS)
    p.set_outcomes(g.integers(0, 2, size=pat.n_meas()).astype(np.uint8))
    x = torch.as_tensor(W.gaussian_state(16, g)).cuda()
    base = pat.angles()
    sets = np.stack([base + g.normal(0, 0.4, base.size) for _ in range(4)])
    l_rev, g_rev = p.adjoint(sets, psi_in=x)
    l_rev, g_rev = l_rev.cpu().numpy(), g_rev.cpu().numpy()
    assert p.plan_info()[2] < p.plan_info()[1]  # tile passes were formed
    l_rec, g_rec = p.adjoint(sets, psi_in=x, ckpt_stride=-8)
    l_rec, g_rec = l_rec.cpu().numpy(), g_rec.cpu().numpy()
    assert np.max(np.abs(l_rev - l_rec)) <= 1e-5
    d = np.abs(g_rev - g_rec)
    assert np.all(d <= 1e-4 * np.maximum(1.0, np.abs(g_rec))), d.max()
    # shift rule on the GPU's own forward losses at sampled (set, angle)
    picks = [(int(g.integers(4)), int(g.integers(base.size))) for _ in range(12)]
    shifted = []
    for b, k in picks:
        for sgn in (1, -1):
            a = sets[b].copy()
            a[k] += sgn * math.pi / 2
            shifted.append(a)
    sl, _ = p.adjoint(np.stack(shifted), psi_in=x)
    sl = sl.cpu().numpy()
    worst = 0.0
    for i, (b, k) in enumerate(picks):
        gs = 0.5 * (sl[2 * i] - sl[2 * i + 1])
        worst = max(worst, abs(gs - g_rev[b, k]))
        assert abs(gs - g_rev[b, k]) <= 1e-4 * max(1.0, abs(gs)), (b, k, gs, g_rev[b, k])
    parity_report("adjoint_masked_windows_width16", max_grad_diff_vs_recompute=float(d.max()),
                  max_grad_diff_vs_gpu_shift=worst)
    p.close()
