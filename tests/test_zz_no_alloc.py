"""GPU checks of the allocation-free entry point (owqs_run_noalloc) against
owqs_run + owqs_read_state + owqs_read_probs on the same patterns.

Several calls in a row share the library's one working array, each smaller
than the one before (a fused plan at live width 21, a plain plan at width 16,
a pattern that runs in one workgroup's LDS at width 10), so a value left by
the previous call must not leak into the next.  Bar: amplitudes within 1e-5,
probabilities within 1e-12 (the same kernels run in the same order).
"""
import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
owqs = pytest.importorskip("paper_1604_05659_amd")

AMP_TOL = 1e-5
NO_ERROR = 0x7FFFFFFF


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return owqs.Context(0)


CASES = [
    # (workload, exec): each narrower than the one before
    (lambda: W.plain_large(index=5, n_logical=20, n_j=150, n_cz=25), owqs.EXEC_FUSED),
    (lambda: W.plain_large(index=6, n_logical=15, n_j=120, n_cz=20), owqs.EXEC_PLAIN),
    (lambda: W.plain_large(index=7, n_logical=9, n_j=80, n_cz=12), owqs.EXEC_AUTO),
]


def _loaded(ctx, wl, exec_):
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_OWQS)
    p.set_exec(exec_)
    p.set_outcomes(wl.outcomes)
    return p


def test_noalloc_matches_run_on_calls_in_a_row(ctx, parity_report):
    loaded = []
    for make, exec_ in CASES:
        wl = make()
        p = _loaded(ctx, wl, exec_)
        x = torch.as_tensor(wl.input_state).cuda()
        p.run(x)                      # uploads the plan; the reference run
        ref = p.read_state().clone()
        ref_p = p.read_probs()
        loaded.append((wl, p, x, ref, ref_p))
    torch.cuda.synchronize()
    widths = [p.max_live for _, p, _, _, _ in loaded]
    assert widths == sorted(widths, reverse=True) and widths[0] == 21
    for rep in range(2):
        for k, (wl, p, x, ref, ref_p) in enumerate(loaded):
            print(f"noalloc call: case {k}, live width {p.max_live}, rep {rep}", flush=True)
            out = torch.full_like(ref, float("nan"))
            probs = torch.full((p.n_meas,), -1.0, dtype=torch.float64, device="cuda")
            err = torch.zeros(2, dtype=torch.int32, device="cuda")
            p.run_noalloc(x, out, probs, err)
            torch.cuda.synchronize()
            d = float((out - ref).abs().max().item())
            pd = float(np.max(np.abs(probs.cpu().numpy() - ref_p)))
            parity_report(f"noalloc_case{k}_rep{rep}", max_amp_diff_vs_run=d, max_p_diff=pd,
                          bit_exact=bool(torch.equal(out, ref)))
            assert d <= AMP_TOL, (k, d)
            assert pd <= 1e-12, (k, pd)
            assert err.cpu().tolist() == [NO_ERROR, 0], k
    # the first case against the oracle as well
    wl, p, _, _, _ = loaded[0]
    want, pw = oc.run(wl.pattern, wl.outcomes, wl.input_state.astype(np.complex128))
    out = torch.empty(1 << p.n_out, dtype=torch.complex64, device="cuda")
    p.run_noalloc(loaded[0][2], out)
    got = out.cpu().numpy().astype(np.complex128)
    assert float(np.max(np.abs(got - want))) <= AMP_TOL
    for _, p, _, _, _ in loaded:
        p.close()


def test_noalloc_reports_zero_probability(ctx):
    """A forced outcome of probability 0 (|+> measured at angle 0 with
    outcome 1) is reported in the caller's error word: index 0 (the M of the
    plain plan, the item of the one-workgroup run) and kind 1."""
    bad = W.Pattern([], [1], [("N", 0), ("N", 1), ("M", 0, 0.0, (), ())])
    for exec_ in (owqs.EXEC_PLAIN, owqs.EXEC_AUTO):
        p = owqs.Pattern(ctx, bad)
        p.set_mode(owqs.MODE_OWQS)
        p.set_exec(exec_)
        p.set_outcomes([1])
        p.run(None)
        with pytest.raises(owqs.OwqsError):
            p.check()
        out = torch.empty(1 << p.n_out, dtype=torch.complex64, device="cuda")
        err = torch.zeros(2, dtype=torch.int32, device="cuda")
        p.run_noalloc(None, out, None, err)
        torch.cuda.synchronize()
        assert err.cpu().tolist() == [0, 1], exec_
        p.close()


def test_noalloc_rejects_stale_plan(ctx):
    wl = W.plain_small()
    p = _loaded(ctx, wl, owqs.EXEC_PLAIN)
    out = torch.empty(1 << p.n_out, dtype=torch.complex64, device="cuda")
    with pytest.raises(owqs.OwqsError) as e:
        p.run_noalloc(None, out)          # never run: no plan on the device
    assert e.value.status == owqs.E_STATE
    p.run(None)
    p.run_noalloc(None, out)
    p.set_outcomes(1 - np.asarray(wl.outcomes))
    with pytest.raises(owqs.OwqsError) as e:
        p.run_noalloc(None, out)          # outcomes changed since the upload
    assert e.value.status == owqs.E_STATE
    torch.cuda.synchronize()
    p.close()
