"""GPU parity on degenerate patterns and calls, against the FP64 oracle:
no commands (identity, with a permuted output order), no inputs, no outputs
(every qubit measured: a single amplitude), a ranged run over no commands,
and empty batch / basis calls.  Tolerance 1e-5 per amplitude."""
import math

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
owqs = pytest.importorskip("paper_1604_05659_amd")

AMP_TOL = 1e-5
EXECS = [owqs.EXEC_PLAIN, owqs.EXEC_FUSED, owqs.EXEC_AUTO]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return owqs.Context(0)


def _run(ctx, pat, outcomes, inp, ex, mode=owqs.MODE_OWQS):
    p = owqs.Pattern(ctx, pat)
    p.set_mode(mode)
    p.set_exec(ex)
    p.set_outcomes(np.asarray(outcomes, np.uint8))
    p.run(None if inp is None else torch.as_tensor(inp).cuda())
    out = p.read_state().cpu().numpy().astype(np.complex128)
    probs = p.read_probs()
    p.close()
    return out, probs


@pytest.mark.parametrize("ex", EXECS)
def test_no_commands_is_the_identity_with_output_order(ctx, ex):
    g = np.random.default_rng(5)
    inp = W.gaussian_state(5, g)
    for outs in ([0, 1, 2, 3, 4], [3, 0, 4, 1, 2]):
        pat = W.Pattern([0, 1, 2, 3, 4], outs, [])
        got, _ = _run(ctx, pat, [], inp, ex)
        want, _ = oc.run(pat, [], inp.astype(np.complex128))
        assert float(np.max(np.abs(got - want))) <= AMP_TOL
    # the permuted order really moves bits: |x> -> |y> with y_k = x_{outs[k]}
    assert not np.allclose(want, inp.astype(np.complex128))


@pytest.mark.parametrize("ex", EXECS)
def test_no_inputs_prepares_plus_states(ctx, ex):
    pat = W.Pattern([], [0, 1, 2], [("N", 0), ("N", 1), ("N", 2), ("E", 0, 2)])
    got, _ = _run(ctx, pat, [], None, ex)
    want, _ = oc.run(pat, [])
    assert float(np.max(np.abs(got - want))) <= AMP_TOL
    assert abs(np.vdot(got, got).real - 1.0) <= 1e-6


@pytest.mark.parametrize("ex", EXECS)
@pytest.mark.parametrize("mode", [owqs.MODE_OWQS, owqs.MODE_EOWQS])
def test_every_qubit_measured_leaves_one_amplitude(ctx, ex, mode):
    g = np.random.default_rng(9)
    cmds = [("N", 2), ("E", 0, 2), ("E", 1, 2), ("M", 0, 0.4, (), ()), ("M", 1, 1.3, (0,), ()),
            ("M", 2, 2.2, (1,), (0,))]
    pat = W.Pattern([0, 1], [], cmds)
    inp = W.gaussian_state(2, g)
    outc = [1, 0, 1]
    got, probs = _run(ctx, pat, outc, inp, ex, mode)
    assert got.shape == (1,)
    if mode == owqs.MODE_OWQS:
        want, pw = oc.run(pat, outc, inp.astype(np.complex128))
        assert float(np.max(np.abs(got - want))) <= AMP_TOL
        np.testing.assert_allclose(probs, pw, atol=1e-6)
        assert abs(abs(got[0]) - 1.0) <= 1e-6


def test_ranged_run_over_no_commands_returns_the_input(ctx):
    g = np.random.default_rng(3)
    wl = W.plain_large(n_logical=6, n_j=10, n_cz=3)
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_outcomes(wl.outcomes)
    x = torch.as_tensor(wl.input_state).cuda()
    p.run_range(0, 0, x)
    live, qubits = p.read_live()
    assert qubits == list(wl.pattern.inputs)
    assert float(np.max(np.abs(live - wl.input_state))) == 0.0
    p.close()


def test_empty_batch_and_basis_calls(ctx):
    owqs.run_batch(ctx, [], [], [])
    wl = W.recognition(n_logical=4, n_j=12, n_cz=3)
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_EOWQS)
    p.set_outcomes(wl.outcomes)
    out = torch.zeros(1, dtype=torch.complex64, device="cuda")
    assert owqs._lib.owqs_run_basis(p._h, 0, 0, out.data_ptr(), None, None) == owqs.OK
    assert owqs._lib.owqs_run_basis(p._h, 0, 0, None, None, None) == owqs.E_INVALID_ARG
    torch.cuda.synchronize()
    p.close()
