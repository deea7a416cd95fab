"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance: max |amplitude error| <= 1e-5 against the complex128 oracle on the
same complex64 inputs (the precision target for complex64 amplitudes with
FP32 arithmetic); FP64 outcome probabilities within 1e-5.
"""
import math

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc
from oracle import reference as ref

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-5
P_TOL = 1e-5

torch = pytest.importorskip("torch")
owqs = pytest.importorskip("paper_1604_05659_amd")

MODES = {"owqs": owqs.MODE_OWQS, "eowqs": owqs.MODE_EOWQS}
EXECS = {"plain": owqs.EXEC_PLAIN, "fused": owqs.EXEC_FUSED, "auto": owqs.EXEC_AUTO}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return owqs.Context(0)


def gpu(ctx, pattern, outcomes, inp=None, mode=owqs.MODE_OWQS, exec_=owqs.EXEC_FUSED):
    out, probs = owqs.run_pattern(ctx, pattern, outcomes, inp, mode, exec_)
    return out.cpu().numpy().astype(np.complex128), probs


def oracle(pattern, outcomes, inp=None, mode=oc.MODE_OWQS):
    x = None if inp is None else np.asarray(inp, np.complex64).astype(np.complex128)
    return oc.run(pattern, outcomes, x, mode)


def assert_close(got, want, tol=AMP_TOL, what=""):
    err = float(np.max(np.abs(got - want))) if got.size else 0.0
    assert err <= tol, f"{what}: max amplitude error {err:.3e} > {tol}"
    return err


def gaussian(n, seed):
    return W.gaussian_state(n, np.random.default_rng(seed))


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("ex", list(EXECS))
def test_fig8_cnot(ctx, mode, ex):
    cmds = [("N", 3), ("E", 2, 3), ("M", 2, 0.0, (), ()),
            ("N", 4), ("E", 3, 4), ("E", 1, 3), ("M", 3, 0.0, (), ()),
            ("Z", 1, (2,)), ("Z", 4, (2,)), ("X", 4, (3,))]
    pat = W.Pattern([1, 2], [1, 4], cmds)
    for k in range(4):
        inp = W.basis_state(2, k)
        for oc_bits in ((0, 0), (0, 1), (1, 0), (1, 1)):
            got, p = gpu(ctx, pat, oc_bits, inp, MODES[mode], EXECS[ex])
            want, pw = oracle(pat, oc_bits, inp, MODES[mode])
            assert_close(got, want, what=f"cnot in={k} o={oc_bits}")
            if mode == "owqs":
                np.testing.assert_allclose(p, pw, atol=P_TOL)


def _kernel_unit_widths():
    return [1, 2, 3, 4, 5, 6, 7, 9, 12, 16, 20]


def _bits_for(n):
    if n <= 12:
        return list(range(n))
    return sorted({0, 1, 2, 3, 4, 5, 6, n // 2, n - 3, n - 2, n - 1})


@pytest.mark.parametrize("n", _kernel_unit_widths())
def test_measure_every_bit(ctx, n):
    """M at every slot (move-to-top layout for b = top, b = 0 and middle bits),
    both outcomes, OWQS renormalisation, width n -> n-1."""
    g = np.random.default_rng(1000 + n)
    inp = gaussian(n, 2000 + n)
    qs = list(range(n))
    for b in _bits_for(n):
        alpha = float(g.uniform(0, 2 * math.pi))
        o = int(g.integers(2))
        pat = W.Pattern(qs, [q for q in qs if q != b], [("M", b, alpha, (), ())])
        got, p = gpu(ctx, pat, [o], inp, owqs.MODE_OWQS, owqs.EXEC_PLAIN)
        want, pw = oracle(pat, [o], inp)
        assert_close(got, want, what=f"M n={n} b={b}")
        np.testing.assert_allclose(p, pw, atol=P_TOL)


@pytest.mark.parametrize("n", _kernel_unit_widths())
def test_prepare_and_entangle_pairs(ctx, n):
    """N (top slot) then E between every sampled pair, read back without
    measurement of the data qubits (the new qubit is measured at angle 0)."""
    g = np.random.default_rng(3000 + n)
    inp = gaussian(n, 4000 + n)
    qs = list(range(n))
    bits = _bits_for(n)
    pairs = [(u, v) for u in bits for v in bits if u < v]
    if len(pairs) > 24:
        pairs = [pairs[i] for i in g.choice(len(pairs), 24, replace=False)]
    for (u, v) in pairs or [(None, None)]:
        cmds = [("N", n)]
        if u is not None:
            cmds.append(("E", u, v))
        cmds.append(("E", n, int(g.integers(n))))
        cmds.append(("M", n, float(g.uniform(0, 2 * math.pi)), (), ()))
        pat = W.Pattern(qs, qs, cmds)
        for ex in EXECS.values():
            got, p = gpu(ctx, pat, [0], inp, owqs.MODE_OWQS, ex)
            want, pw = oracle(pat, [0], inp)
            assert_close(got, want, what=f"E n={n} ({u},{v})")


@pytest.mark.parametrize("n", _kernel_unit_widths())
def test_pauli_corrections_every_bit(ctx, n):
    """X and Z at every sampled slot, switched on by a signal of 1 taken from
    an auxiliary qubit measured with probability 1."""
    inp = gaussian(n, 5000 + n)
    qs = list(range(n))
    for b in _bits_for(n):
        for op in ("X", "Z"):
            cmds = [("N", n), ("M", n, math.pi, (), ()), (op, b, (n,))]
            pat = W.Pattern(qs, qs, cmds)
            got, p = gpu(ctx, pat, [1], inp, owqs.MODE_OWQS, owqs.EXEC_PLAIN)
            want, pw = oracle(pat, [1], inp)
            assert_close(got, want, what=f"{op} n={n} b={b}")
            assert abs(p[0] - 1.0) < P_TOL


@pytest.mark.parametrize("n", _kernel_unit_widths())
def test_j_window_every_bit(ctx, n):
    """N w; E u w; M u; X w: fused 2x2 pass vs oracle, both outcomes and modes."""
    g = np.random.default_rng(6000 + n)
    inp = gaussian(n, 7000 + n)
    qs = list(range(n))
    for b in _bits_for(n):
        alpha = float(g.uniform(0, 2 * math.pi))
        pat = W.Pattern(qs, [q for q in qs if q != b] + [n],
                        [("N", n), ("E", b, n), ("M", b, alpha, (), ()), ("X", n, (b,)), ("Z", n, (b,))])
        for o in (0, 1):
            for mode in MODES.values():
                for ex in EXECS.values():
                    got, p = gpu(ctx, pat, [o], inp, mode, ex)
                    want, pw = oracle(pat, [o], inp, mode)
                    assert_close(got, want, what=f"J n={n} b={b} o={o} mode={mode} ex={ex}")


@pytest.mark.parametrize("n", [2, 3, 5, 8, 13, 17])
def test_generalized_windows(ctx, n):
    """N w; E's on v or w (to other qubits too, E(v, w) an odd or even number
    of times); M v; X/Z on w: fused windows with index-parity signs."""
    g = np.random.default_rng(8000 + n)
    inp = gaussian(n, 9000 + n)
    qs = list(range(n))
    for trial in range(6):
        v = int(g.integers(n))
        others = [q for q in qs if q != v]
        cmds = [("N", n)]
        es = [("E", v, n)]
        if trial % 3 == 1:
            es.append(("E", n, v))          # E(v, w) twice: they cancel
        elif trial % 3 == 2:
            es += [("E", n, v), ("E", v, n)]  # three times: one CZ
        for x in g.choice(others, size=min(len(others), int(g.integers(0, 3))), replace=False) if others else []:
            es.append(("E", v, int(x)))
        for y in g.choice(others, size=min(len(others), int(g.integers(0, 3))), replace=False) if others else []:
            es.append(("E", n, int(y)))
        g.shuffle(es)
        cmds += [tuple(e) for e in es]
        cmds.append(("M", v, float(g.uniform(0, 2 * math.pi)), (), ()))
        cmds += [("Z", n, (v,)), ("X", n, (v,))] if trial % 2 else [("X", n, (v,))]
        pat = W.Pattern(qs, [q for q in qs if q != v] + [n], cmds)
        for o in (0, 1):
            want, pw = oracle(pat, [o], inp)
            for ex in EXECS.values():
                got, p = gpu(ctx, pat, [o], inp, owqs.MODE_OWQS, ex)
                assert_close(got, want, what=f"window n={n} trial={trial} o={o} ex={ex}")
                np.testing.assert_allclose(p, pw, atol=P_TOL)


def test_random_patterns(ctx):
    g = np.random.default_rng(1604)
    done = 0
    for trial in range(80):
        pat = W.random_pattern(g, max_qubits=int(g.integers(4, 12)))
        nin = len(pat.inputs)
        inp = gaussian(nin, 100 + trial) if nin else None
        outc = g.integers(0, 2, size=pat.n_meas()).astype(np.uint8)
        try:
            want, pw = oracle(pat, outc, inp)
        except oc.OracleError:
            continue
        if pw.size and pw.min() < 1e-4:
            continue
        for ex in EXECS.values():
            got, p = gpu(ctx, pat, outc, inp, owqs.MODE_OWQS, ex)
            assert_close(got, want, what=f"random trial {trial} ex={ex}")
            np.testing.assert_allclose(p, pw, atol=P_TOL)
        done += 1
    assert done >= 40


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("ex", list(EXECS))
def test_plain_small_workload(ctx, mode, ex):
    for idx in range(4):
        wl = W.plain_small(index=idx)
        got, p = gpu(ctx, wl.pattern, wl.outcomes, None, MODES[mode], EXECS[ex])
        want, pw = oracle(wl.pattern, wl.outcomes, None, MODES[mode])
        assert_close(got, want, what=f"plain_small[{idx}]")
        if mode == "owqs":
            np.testing.assert_allclose(p, pw, atol=P_TOL)


@pytest.mark.parametrize("n_logical,n_j,n_cz", [(8, 120, 20), (12, 300, 45), (16, 200, 30)])
@pytest.mark.parametrize("ex", list(EXECS))
def test_plain_large_shape(ctx, n_logical, n_j, n_cz, ex):
    wl = W.plain_large(n_logical=n_logical, n_j=n_j, n_cz=n_cz)
    for mode in MODES.values():
        got, p = gpu(ctx, wl.pattern, wl.outcomes, wl.input_state, mode, EXECS[ex])
        want, pw = oracle(wl.pattern, wl.outcomes, wl.input_state, mode)
        assert_close(got, want, what=f"plain_large {n_logical} mode={mode}")


@pytest.mark.parametrize("rows,cols", [(3, 8), (6, 20), (10, 12)])
@pytest.mark.parametrize("ex", list(EXECS))
def test_cluster_shape(ctx, rows, cols, ex):
    wl = W.cluster(rows=rows, cols=cols)
    got, p = gpu(ctx, wl.pattern, wl.outcomes, None, owqs.MODE_OWQS, EXECS[ex])
    want, pw = oracle(wl.pattern, wl.outcomes)
    assert_close(got, want, what=f"cluster {rows}x{cols}")
    np.testing.assert_allclose(p, pw, atol=P_TOL)


def test_recognition_shape_basis_inputs(ctx):
    wl = W.recognition(n_logical=5, n_j=40, n_cz=8)
    u = ref.circuit_unitary(5, wl.meta["gates"])
    for k in range(32):
        got, _ = gpu(ctx, wl.pattern, wl.outcomes, W.basis_state(5, k), owqs.MODE_EOWQS)
        assert_close(got, u[:, k], what=f"column {k}")


def test_reuse_pattern_between_runs(ctx):
    """Same loaded pattern, several runs with new inputs / outcomes / angles."""
    wl = W.plain_large(n_logical=10, n_j=80, n_cz=10)
    p = owqs.Pattern(ctx, wl.pattern)
    g = np.random.default_rng(5)
    for r in range(4):
        outc = g.integers(0, 2, size=wl.pattern.n_meas()).astype(np.uint8)
        ang = g.uniform(0, 2 * math.pi, size=wl.pattern.n_meas())
        inp = gaussian(10, 50 + r)
        p.set_outcomes(outc)
        p.set_angles(ang)
        p.set_exec(owqs.EXEC_FUSED if r % 2 else owqs.EXEC_PLAIN)
        p.run(torch.as_tensor(inp).cuda())
        got = p.read_state().cpu().numpy().astype(np.complex128)
        want, _ = oracle(wl.pattern.with_angles(ang), outc, inp)
        assert_close(got, want, what=f"run {r}")
    p.close()


def test_zero_probability_is_reported(ctx):
    # |0> measured at angle 0: outcome 1 ... p = 1/2; |+> at angle 0 with outcome 1 has p = 0
    pat = W.Pattern([], [1], [("N", 0), ("N", 1), ("M", 0, 0.0, (), ())])
    p = owqs.Pattern(ctx, pat)
    p.set_outcomes([1])
    p.run(None)
    with pytest.raises(owqs.OwqsError) as e:
        p.read_state()
    assert e.value.status == owqs.E_ZERO_PROB
    p.close()


def test_eowqs_check_flags_non_deterministic(ctx):
    inp = np.array([math.cos(0.3), math.sin(0.3)], np.complex64)
    pat = W.Pattern([0], [], [("M", 0, 0.0, (), ())])
    p = owqs.Pattern(ctx, pat)
    p.set_mode(owqs.MODE_EOWQS_CHECK)
    p.set_outcomes([0])
    p.run(torch.as_tensor(inp).cuda())
    with pytest.raises(owqs.OwqsError) as e:
        p.read_state()
    assert e.value.status == owqs.E_NOT_DETERMINISTIC
    # a flow pattern passes the check
    wl = W.plain_small()
    q = owqs.Pattern(ctx, wl.pattern)
    q.set_mode(owqs.MODE_EOWQS_CHECK)
    q.set_outcomes(wl.outcomes)
    q.run(None)
    got = q.read_state().cpu().numpy()
    want, _ = oracle(wl.pattern, wl.outcomes)
    assert_close(got.astype(np.complex128), want)
    np.testing.assert_allclose(q.read_probs(), 0.5, atol=P_TOL)
    p.close()
    q.close()
