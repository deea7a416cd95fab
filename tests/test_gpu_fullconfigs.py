"""Element-by-element parity with the FP64 oracle at the full sizes of the
workloads, in the launch configurations that bench.py times (the paper
validates its simulator by comparing outputs, Sec. 5).

* plain_large, the whole 8300-command pattern at 2^25 amplitudes, plain and
  fused executors: every outcome probability, the amplitudes at 65 536 seeded
  output indices, <Z_i> of every output qubit and the norm, against values
  the oracle wrote (``tests/golden/make_goldens.py``).
* the 20 x 200 cluster (width 21), plain and fused: all 2^20 output
  amplitudes and every probability, the oracle run here.
* the 512-pattern batch (widths 8..20, 50..800 commands) through one
  owqs_run_batch call: every output amplitude and probability of every
  pattern, the oracle run here.
* the differentiated workload (16 qubits, 25 layers, 64 angle sets): the
  losses and all 400 gradient entries of sets 0 and 1 against the oracle's
  exact shift rule (stored by the same script).

Bars: amplitudes within 1e-5 (complex64 against complex128), probabilities
within 1e-5, gradients within 1e-4 * max(1, |g|).
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
owqs = pytest.importorskip("paper_1604_05659_amd")

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD_PLAIN = os.path.join(HERE, "golden", "plain_large_full.npz")
GOLD_GRAD = os.path.join(HERE, "golden", "ansatz_gradient.npz")
AMP_TOL = 1e-5
P_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return owqs.Context(0)


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def _oracle_many(jobs):
    """Runs independent oracle calls on a thread pool, one OpenMP thread each."""
    def one(job):
        oc.set_threads(1)
        return job()
    with ThreadPoolExecutor(_threads()) as ex:
        return list(ex.map(one, jobs))


def _goldens():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_owqs_goldens", os.path.join(HERE, "golden", "make_goldens.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _fidelity(a, b):
    return abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


def test_plain_large_whole_pattern_against_oracle(ctx, parity_report):
    gold = np.load(GOLD_PLAIN, allow_pickle=False)
    wl = W.plain_large()
    idx = gold["idx"]
    assert np.array_equal(idx, _goldens().sample_indices(len(wl.pattern.outputs))), "golden sample indices"
    assert gold["probs"].size == wl.pattern.n_meas() == 2000
    want = gold["amp"]
    inp = torch.as_tensor(wl.input_state).cuda()
    x = torch.arange(1 << 24, device="cuda")
    for ex, name in ((owqs.EXEC_PLAIN, "plain"), (owqs.EXEC_FUSED, "fused")):
        print(f"plain_large full pattern, {name} executor", flush=True)
        p = owqs.Pattern(ctx, wl.pattern)
        p.set_mode(owqs.MODE_OWQS)
        p.set_exec(ex)
        p.set_outcomes(wl.outcomes)
        p.run(inp)
        out = p.read_state()
        probs = p.read_probs()
        p2 = (out.real.double() ** 2 + out.imag.double() ** 2)
        z = np.array([float((p2 * (1 - 2 * ((x >> i) & 1)).double()).sum()) for i in range(24)])
        norm = float(p2.sum().sqrt())
        got = out[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
        torch.cuda.synchronize()
        p.close()
        err = float(np.max(np.abs(got - want)))
        perr = float(np.max(np.abs(probs - gold["probs"])))
        zerr = float(np.max(np.abs(z - gold["z"])))
        parity_report(f"plain_large_full_oracle_{name}", max_amp_err_sampled=err, samples=int(idx.size),
                      max_p_err=perr, max_z_err=zerr, one_minus_fidelity_sampled=1.0 - _fidelity(got, want))
        assert err <= AMP_TOL, (name, err)
        assert perr <= P_TOL, (name, perr)
        assert zerr <= 1e-5, (name, zerr)
        assert abs(norm - float(gold["norm"])) <= 1e-5, (name, norm)


@pytest.fixture(scope="module")
def cluster_oracle():
    wl = W.cluster()
    oc.set_threads(_threads())
    psi, probs = oc.run(wl.pattern, wl.outcomes)
    return wl, psi, probs


@pytest.mark.parametrize("exec_,name", [(owqs.EXEC_PLAIN, "plain"), (owqs.EXEC_FUSED, "fused")])
def test_cluster_20x200_all_outputs(ctx, cluster_oracle, exec_, name, parity_report):
    wl, want, pw = cluster_oracle
    print(f"cluster 20x200, {name} executor", flush=True)
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_OWQS)
    p.set_exec(exec_)
    p.set_outcomes(wl.outcomes)
    p.run(None)
    got = p.read_state().cpu().numpy().astype(np.complex128)
    probs = p.read_probs()
    p.close()
    assert got.size == want.size == 1 << 20
    err = float(np.max(np.abs(got - want)))
    perr = float(np.max(np.abs(probs - pw)))
    parity_report(f"cluster_20x200_full_{name}", max_amp_err=err, max_p_err=perr,
                  one_minus_fidelity=1.0 - _fidelity(got, want))
    assert err <= AMP_TOL, err
    assert perr <= P_TOL, perr


def test_batch_512_patterns_against_oracle(ctx, parity_report):
    wls = [W.batched_random(i) for i in range(512)]
    pats, ins, outs = [], [], []
    for wl in wls:
        p = owqs.Pattern(ctx, wl.pattern)
        p.set_mode(owqs.MODE_OWQS)
        p.set_outcomes(wl.outcomes)
        pats.append(p)
        ins.append(torch.as_tensor(wl.input_state).cuda())
        outs.append(torch.empty(1 << len(wl.pattern.outputs), dtype=torch.complex64, device="cuda"))
    widths = [p.plan_info()[0] for p in pats]
    print(f"512-pattern batch, plan widths {min(widths)}..{max(widths)}", flush=True)
    wants = _oracle_many([
        (lambda wl=wl: oc.run(wl.pattern, wl.outcomes, wl.input_state.astype(np.complex128)))
        for wl in wls])
    for rep in range(2):
        for o in outs:
            o.fill_(float("nan"))
        owqs.run_batch(ctx, pats, ins, outs)
        torch.cuda.synchronize()
        worst, pworst = 0.0, 0.0
        for k, (p, o) in enumerate(zip(pats, outs)):
            p.check()
            want, pw = wants[k]
            got = o.cpu().numpy().astype(np.complex128)
            e = float(np.max(np.abs(got - want)))
            pe = float(np.max(np.abs(p.read_probs() - pw))) if pw.size else 0.0
            assert e <= AMP_TOL, (k, widths[k], e)
            assert pe <= P_TOL, (k, widths[k], pe)
            worst, pworst = max(worst, e), max(pworst, pe)
        parity_report(f"batched_random_512_rep{rep}", max_amp_err=worst, max_p_err=pworst)
    for p in pats:
        p.close()


def test_ansatz_full_gradient_against_oracle(ctx, parity_report):
    gold = np.load(GOLD_GRAD, allow_pickle=False)
    wl, sets = W.ansatz()
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_EOWQS)
    p.set_outcomes(wl.outcomes)
    loss, grad = p.adjoint(sets)
    loss, grad = loss.cpu().numpy(), grad.cpu().numpy()
    p.close()
    worst = 0.0
    for b in gold["sets"]:
        b = int(b)
        g = gold[f"grad{b}"]
        assert g.size == 400
        assert abs(loss[b] - float(gold[f"loss{b}"])) <= 1e-5
        d = np.abs(grad[b] - g)
        assert np.all(d <= 1e-4 * np.maximum(1.0, np.abs(g))), (b, float(d.max()))
        worst = max(worst, float(d.max()))
    parity_report("adjoint_full_gradient_sets_0_1", max_abs_grad_err=worst, entries=400 * len(gold["sets"]))
