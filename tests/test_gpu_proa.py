"""GPU parity of reordered patterns (PROA, Sec. 4.3): a standard-form
pattern, reordered by the library (owqs_pattern_reorder), runs on the device
and gives the oracle's output state and joint outcome probability for the
source pattern.  Tolerances as in the other parity tests: 1e-5 on complex64
amplitudes; the joint probability (the product of the per-M conditionals,
which depend on the order) to 1e-4 relative."""
import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-5

torch = pytest.importorskip("torch")
owqs = pytest.importorskip("paper_1604_05659_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return owqs.Context(0)


def per_qubit(pattern, outcomes):
    return dict(zip([c[1] for c in pattern.cmds if c[0] == "M"], (int(b) for b in outcomes)))


def outcomes_of(pattern, per_q):
    return np.array([per_q[c[1]] for c in pattern.cmds if c[0] == "M"], np.uint8)


def run_gpu(p, outcomes, inp, mode, exec_=owqs.EXEC_AUTO):
    p.set_mode(mode)
    p.set_exec(exec_)
    p.set_outcomes(outcomes)
    p.run(None if inp is None else torch.as_tensor(inp.astype(np.complex64)).cuda())
    out = p.read_state().cpu().numpy().astype(np.complex128)
    return out, p.read_probs()


@pytest.mark.parametrize("rows,cols", [(4, 10), (8, 30), (12, 16), (20, 12)])
def test_reordered_cluster_against_oracle(ctx, rows, cols):
    wl = W.cluster(rows=rows, cols=cols)
    std = W.standard_form(wl.pattern)
    src = owqs.Pattern(ctx, std)
    re, stats = src.reorder()
    assert stats["max_state_space"] == rows + 1
    spec = re.commands()
    per_q = per_qubit(wl.pattern, wl.outcomes)
    print(f"[proa] cluster {rows}x{cols} live {stats['max_live']}", flush=True)
    want, pw = oc.run(wl.pattern, wl.outcomes)
    for ex in (owqs.EXEC_PLAIN, owqs.EXEC_FUSED):
        got, pg = run_gpu(re, outcomes_of(spec, per_q), None, owqs.MODE_OWQS, ex)
        assert np.max(np.abs(got - want)) <= AMP_TOL, (rows, cols, ex)
        assert float(np.prod(pg)) == pytest.approx(float(np.prod(pw)), rel=1e-4)
    re.close()
    src.close()


def test_reordered_random_patterns_against_oracle(ctx):
    g = np.random.default_rng(4501)
    for i in range(24):
        pat = W.random_standard_pattern(g, n_qubits=int(g.integers(6, 17)), n_in=int(g.integers(0, 4)),
                                        n_out=int(g.integers(1, 4)), extra_edges=int(g.integers(0, 8)),
                                        max_dom=int(g.integers(0, 3)))
        src = owqs.Pattern(ctx, pat)
        re, stats = src.reorder()
        spec = re.commands()
        per_q = {c[1]: int(g.integers(2)) for c in pat.cmds if c[0] == "M"}
        inp = W.gaussian_state(len(pat.inputs), g) if pat.inputs else None
        print(f"[proa] random {i} qubits {len({c[1] for c in pat.cmds})} live {stats['max_live']}", flush=True)
        want, pw = oc.run(pat, outcomes_of(pat, per_q), None if inp is None else inp.astype(np.complex128))
        got, pg = run_gpu(re, outcomes_of(spec, per_q), inp, owqs.MODE_OWQS)
        assert np.max(np.abs(got - want)) <= AMP_TOL, i
        assert float(np.prod(pg)) == pytest.approx(float(np.prod(pw)), rel=1e-4)
        re.close()
        src.close()


@pytest.mark.parametrize("rows,cols", [(5, 14), (16, 12)])
def test_positive_branch_eowqs(ctx, rows, cols):
    """EOWQS on the positive branch (Sec. 4.5): dependencies ignored, every
    outcome 0, fixed scale; equals the source pattern's all-zero branch."""
    wl = W.cluster(rows=rows, cols=cols)
    std = W.standard_form(wl.pattern)
    src = owqs.Pattern(ctx, std)
    re, stats = src.reorder(ignore_dependencies=True)
    spec = re.commands()
    assert all(not c[3] and not c[4] for c in spec.cmds if c[0] == "M")
    assert not any(c[0] in ("X", "Z") for c in spec.cmds)
    zeros = np.zeros(re.n_meas, np.uint8)
    got, _ = run_gpu(re, zeros, None, owqs.MODE_EOWQS)
    want, _ = oc.run(wl.pattern, np.zeros(wl.pattern.n_meas(), np.uint8), None, oc.MODE_EOWQS)
    assert np.max(np.abs(got - want)) <= AMP_TOL
    re.close()
    src.close()


def test_full_size_cluster_reordered_matches_column_order(ctx):
    """20 x 200 cluster: the standard form (4000 qubits, too wide to run)
    reordered by the library runs at the width of the column-by-column
    pattern and gives its output; that pattern is checked against the oracle
    at smaller sizes.  Properties at full size: same state within 1e-5, unit
    norm, same joint probability."""
    wl = W.cluster(rows=20, cols=200)
    std = W.standard_form(wl.pattern)
    src = owqs.Pattern(ctx, std)
    assert src.max_live > owqs.MAX_WIDTH
    re, stats = src.reorder()
    assert stats["max_state_space"] == 21 and stats["max_live"] <= 22
    spec = re.commands()
    per_q = per_qubit(wl.pattern, wl.outcomes)
    got, pg = run_gpu(re, outcomes_of(spec, per_q), None, owqs.MODE_OWQS, owqs.EXEC_FUSED)
    col = owqs.Pattern(ctx, wl.pattern)
    want, pw = run_gpu(col, wl.outcomes, None, owqs.MODE_OWQS, owqs.EXEC_FUSED)
    assert np.max(np.abs(got - want)) <= AMP_TOL
    assert abs(np.linalg.norm(got) - 1.0) <= 1e-5
    assert float(np.sum(np.log(pg))) == pytest.approx(float(np.sum(np.log(pw))), abs=1e-3)
    col.close()
    re.close()
    src.close()
