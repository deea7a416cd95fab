"""GPU check of the EOWQS certificate (owqs_pattern_certify, Sec. 4.5): on
random XY-plane patterns, a fully certified pattern passes the device's
EOWQS_CHECK mode (every p within 1e-4 of 1/2) and its EOWQS output equals the
OWQS output within 1e-5; a pattern whose oracle probabilities leave 1/2 at an
uncertified measurement is flagged by the device (OWQS_E_NOT_DETERMINISTIC)."""
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


def random_xy_pattern(g, n, p_edge):
    qs = list(range(n))
    n_in = int(g.integers(0, 3))
    n_out = int(g.integers(1, 3))
    perm = list(g.permutation(n))
    ins, outs = sorted(perm[:n_in]), sorted(perm[n - n_out:])
    edges = {(a, b) for a in qs for b in qs if a < b and g.random() < p_edge}
    cmds = [("N", q) for q in qs if q not in ins] + [("E", a, b) for a, b in sorted(edges)]
    meas = [q for q in g.permutation(n).tolist() if q not in outs]
    done = []
    for q in meas:
        k = int(g.integers(0, min(2, len(done)) + 1))
        s = tuple(int(x) for x in g.choice(done, size=k, replace=False)) if k else ()
        cmds.append(("M", q, float(g.uniform(0, 2 * math.pi)), s, ()))
        done.append(q)
    return W.Pattern(ins, outs, cmds)


def test_certified_patterns_pass_the_device_check(ctx):
    g = np.random.default_rng(5101)
    certified = flagged = 0
    for i in range(200):
        pat = random_xy_pattern(g, int(g.integers(3, 13)), float(g.uniform(0.2, 0.6)))
        if i % 3 == 0:
            # a flow pattern: a J/CZ circuit (certified by construction)
            nl = int(g.integers(2, 6))
            pat = W.circuit_to_pattern(nl, W.random_jcz_circuit(nl, int(g.integers(3, 20)), int(g.integers(1, 5)), g))
        elif i % 3 == 1:
            # measure in the order of a gflow's layers, when there is one
            q = owqs.Pattern(ctx, pat)
            ex, _, layer = q.gflow()
            q.close()
            if ex:
                ms = [c for c in pat.cmds if c[0] == "M"]
                ms = [m for _, m in sorted(zip(-layer, range(len(ms))), key=lambda t: t[0])]
                order = [[c for c in pat.cmds if c[0] == "M"][k] for k in ms]
                # domains must stay on earlier measurements: drop them (angles are free)
                order = [("M", c[1], c[2], (), ()) for c in order]
                pat = W.Pattern(pat.inputs, pat.outputs, [c for c in pat.cmds if c[0] != "M"] + order)
        inp = W.gaussian_state(len(pat.inputs), g) if pat.inputs else None
        if inp is not None:
            inp = (inp / np.linalg.norm(inp)).astype(np.complex64)
        outc = g.integers(0, 2, pat.n_meas()).astype(np.uint8)
        try:
            _, pw = oc.run(pat, outc, None if inp is None else inp.astype(np.complex128))
        except oc.OracleError:
            continue
        if len(pw) and pw.min() < 1e-3:
            continue
        p = owqs.Pattern(ctx, pat)
        ok, first = p.certify()
        p.set_outcomes(outc)
        dev_in = None if inp is None else torch.as_tensor(inp).cuda()
        p.set_mode(owqs.MODE_EOWQS_CHECK)
        p.run(dev_in)
        if ok.all():
            certified += 1
            got = p.read_state().cpu().numpy()       # raises if the device flagged a p
            np.testing.assert_allclose(p.read_probs(), 0.5, atol=1e-5)
            p.set_mode(owqs.MODE_OWQS)
            p.run(dev_in)
            want = p.read_state().cpu().numpy()
            assert np.max(np.abs(got - want)) <= 1e-5, i
        elif np.max(np.abs(pw - 0.5)) > 1e-3:
            flagged += 1
            with pytest.raises(owqs.OwqsError) as e:
                p.read_state()
            assert e.value.status == owqs.E_NOT_DETERMINISTIC
            # every certified M before the first uncertified one is exactly 1/2
            assert np.allclose(pw[:first], 0.5, atol=1e-6)
        p.close()
    assert certified >= 30 and flagged >= 30
