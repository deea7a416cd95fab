"""Parity at the full size of the large plain workload (24 logical qubits,
live width 24 <-> 25, 2^25 amplitudes) in the launch configuration that
bench.py times.

* element by element against the FP64 oracle on a prefix of the circuit
  (the oracle finishes it in seconds at this width);
* on the whole 8300-command pattern, properties that hold at any size: every
  outcome probability is 1/2 (the pattern has a flow), the output has norm 1,
  plain and fused executors agree, another outcome string gives the same
  output (determinism), and the pattern followed by the pattern of the
  inverse circuit returns the input state.
"""
import os

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


@pytest.fixture(scope="module")
def large():
    return W.plain_large()


def _run(ctx, pattern, outcomes, inp, exec_, mode=owqs.MODE_OWQS):
    p = owqs.Pattern(ctx, pattern)
    p.set_mode(mode)
    p.set_exec(exec_)
    p.set_outcomes(outcomes)
    p.run(inp)
    out = p.read_state()
    probs = p.read_probs()
    torch.cuda.synchronize()
    p.close()
    return out, probs


def _fidelity(a, b):
    a = a.astype(np.complex128)
    b = b.astype(np.complex128)
    return abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


def test_full_width_prefix_against_oracle(ctx, large, parity_report):
    gates = large.meta["gates"][:20]
    pat = W.circuit_to_pattern(24, gates)
    outc = W.outcome_bits(pat.n_meas(), np.random.default_rng(77))
    oc.set_threads(os.cpu_count() or 1)
    want, pw = oc.run(pat, outc, large.input_state.astype(np.complex128))
    inp = torch.as_tensor(large.input_state).cuda()
    for ex, name in ((owqs.EXEC_PLAIN, "plain"), (owqs.EXEC_FUSED, "fused")):
        out, probs = _run(ctx, pat, outc, inp, ex)
        got = out.cpu().numpy().astype(np.complex128)
        err = float(np.max(np.abs(got - want)))
        one_minus_f = 1.0 - _fidelity(got, want)
        parity_report(f"plain_large_prefix20_{name}", max_amp_err=err, one_minus_fidelity=one_minus_f,
                      max_p_err=float(np.max(np.abs(probs - pw))))
        assert err <= AMP_TOL, err
        assert one_minus_f <= 1e-9, one_minus_f
        np.testing.assert_allclose(probs, pw, atol=1e-6)


def test_full_pattern_properties(ctx, large, parity_report):
    inp = torch.as_tensor(large.input_state).cuda()
    out_p, probs_p = _run(ctx, large.pattern, large.outcomes, inp, owqs.EXEC_PLAIN)
    out_f, probs_f = _run(ctx, large.pattern, large.outcomes, inp, owqs.EXEC_FUSED)
    other = W.outcome_bits(large.pattern.n_meas(), np.random.default_rng(123))
    out_o, _ = _run(ctx, large.pattern, other, inp, owqs.EXEC_FUSED)
    a, b, c = (t.cpu().numpy().astype(np.complex128) for t in (out_p, out_f, out_o))
    assert np.max(np.abs(probs_p - 0.5)) <= 1e-5
    assert np.max(np.abs(probs_f - 0.5)) <= 1e-5
    assert abs(np.linalg.norm(a) - 1) <= 1e-5 and abs(np.linalg.norm(b) - 1) <= 1e-5
    d_pf = float(np.max(np.abs(a - b)))
    d_det = float(np.max(np.abs(b - c)))
    parity_report("plain_large_full_plain_vs_fused", max_amp_diff=d_pf, one_minus_fidelity=1 - _fidelity(a, b))
    parity_report("plain_large_full_other_outcomes", max_amp_diff=d_det, one_minus_fidelity=1 - _fidelity(b, c))
    assert d_pf <= AMP_TOL and d_det <= AMP_TOL


def test_full_pattern_then_inverse_returns_input(ctx, large, parity_report):
    gates = large.meta["gates"]
    pat = W.circuit_to_pattern(24, gates + W.inverse_jcz_gates(gates))
    outc = W.outcome_bits(pat.n_meas(), np.random.default_rng(5))
    inp = torch.as_tensor(large.input_state).cuda()
    x = large.input_state.astype(np.complex128)
    for ex, name in ((owqs.EXEC_FUSED, "fused"), (owqs.EXEC_PLAIN, "plain")):
        out, probs = _run(ctx, pat, outc, inp, ex)
        got = out.cpu().numpy().astype(np.complex128)
        err = float(np.max(np.abs(got - x)))
        one_minus_f = 1 - _fidelity(got, x)
        parity_report(f"plain_large_forward_inverse_{name}", max_amp_err=err, one_minus_fidelity=one_minus_f,
                      commands=len(pat.cmds))
        assert err <= AMP_TOL, err
        assert one_minus_f <= 1e-8, one_minus_f
        assert np.max(np.abs(probs - 0.5)) <= 1e-5


@pytest.mark.parametrize("nl", [25, 26])
def test_plain_kernels_above_the_cache_against_oracle(ctx, nl, parity_report):
    """Live widths nl <-> nl + 1 (2^26 and 2^27 amplitudes, above the 256 MB
    Infinity Cache), where N, M and X stream with the non-temporal hint: a
    short circuit element by element against the FP64 oracle."""
    g = np.random.default_rng([160405659, 11, 0, nl])
    pat = W.circuit_to_pattern(nl, W.random_jcz_circuit(nl, 4, 2, g))
    outc = g.integers(0, 2, pat.n_meas()).astype(np.uint8)
    inp = W.gaussian_state(nl, g)
    print(f"[fullsize] width {nl}<->{nl + 1}, {len(pat.cmds)} commands", flush=True)
    got, probs = _run(ctx, pat, outc, torch.as_tensor(inp).cuda(), owqs.EXEC_PLAIN)
    got = got.cpu().numpy().astype(np.complex128)
    want, pw = oc.run(pat, outc, inp.astype(np.complex128))
    err = float(np.max(np.abs(got - want)))
    parity_report(f"plain kernels at 2^{nl + 1}", max_err=err, infidelity=1 - _fidelity(got, want))
    assert err <= AMP_TOL
    np.testing.assert_allclose(probs, pw, atol=1e-5)


@pytest.mark.parametrize("nl", [28, 29])
def test_fused_at_the_buffer_offset_boundary(ctx, nl, parity_report):
    """Tile passes at live width 28, the widest that moves its tiles through
    buffer loads and stores (byte offsets up to 2^31 - 8), and at 29 (64-bit
    global addresses; a buffer's record count, 2^32 - 1 bytes at most, would
    leave the last dword of the vector out of range there): a short circuit
    run fused and plain on the same seeded input, compared element by
    element on the device (2^nl amplitudes, beyond what the oracle holds;
    the plain kernels are checked against the oracle at every width above)."""
    g = np.random.default_rng([160405659, 12, 0, nl])
    pat = W.circuit_to_pattern(nl, W.random_jcz_circuit(nl, 4, 2, g))
    outc = g.integers(0, 2, pat.n_meas()).astype(np.uint8)
    gen = torch.Generator(device="cuda").manual_seed(160405659 + nl)
    inp = torch.randn(1 << nl, dtype=torch.complex64, device="cuda", generator=gen)
    inp /= torch.linalg.vector_norm(inp)
    print(f"[fullsize] fused at width {nl}<->{nl + 1}, {len(pat.cmds)} commands", flush=True)
    out_f, pf = _run(ctx, pat, outc, inp, owqs.EXEC_FUSED)
    out_p, pp = _run(ctx, pat, outc, inp, owqs.EXEC_PLAIN)
    err = float((out_f - out_p).abs().max().item())
    norm = float(torch.linalg.vector_norm(out_f).item())
    parity_report(f"fused vs plain at 2^{nl}", max_err=err, norm=norm)
    assert err <= AMP_TOL, err
    assert abs(norm - 1.0) <= 1e-4, norm
    np.testing.assert_allclose(pf, pp, atol=1e-6)
