"""Writes the stored expected values of the full-size parity tests.

Every value here comes from the FP64 oracle (``oracle/``) run on the seeded
workloads of ``owqs_workloads``; nothing is taken from the GPU library.

    python tests/golden/make_goldens.py plain_large   # plain_large_full.npz
    python tests/golden/make_goldens.py gradient      # ansatz_gradient.npz

plain_large: the whole 8300-command pattern of the large plain workload
(24 logical qubits, 2000 J + 300 CZ, live width 24 <-> 25) on its complex
Gaussian input (the complex64-rounded values, upcast), with its seeded forced
outcomes, in OWQS mode.  Stored: every outcome probability (Eq. 13), the
output amplitudes at a seeded sample of 65 536 output indices, <Z_i> of every
output qubit over the whole output (a property of all 2^24 amplitudes), the
output's norm, and the oracle's wall time and thread count.

gradient: the differentiated workload (16 logical qubits, 25 layers, 400
angles), angle sets 0 and 1: the loss sum_i <Z_i> and all 400 entries of
dL/d(alpha) by the exact two-term shift rule (EOWQS; Eqs. 2, 11-12), 800
oracle forwards per set.
"""
import os
import platform
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import owqs_workloads as W  # noqa: E402
from oracle import core as oc  # noqa: E402

PLAIN_LARGE = os.path.join(HERE, "plain_large_full.npz")
GRADIENT = os.path.join(HERE, "ansatz_gradient.npz")
N_SAMPLE = 1 << 16


def sample_indices(nout: int, count: int = N_SAMPLE) -> np.ndarray:
    """Seeded output indices of the plain_large sample (purpose 9 of config 2)."""
    g = W.rng(2, 9, 0)
    return np.sort(g.choice(1 << nout, size=count, replace=False)).astype(np.int64)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def plain_large() -> None:
    wl = W.plain_large()
    threads = oc.set_threads(os.cpu_count() or 1)
    inp = wl.input_state.astype(np.complex128)
    t0 = time.perf_counter()
    psi, probs = oc.run(wl.pattern, wl.outcomes, inp, oc.MODE_OWQS)
    wall = time.perf_counter() - t0
    nout = len(wl.pattern.outputs)
    idx = sample_indices(nout)
    p2 = np.abs(psi) ** 2
    x = np.arange(1 << nout)
    z = np.array([np.sum(p2 * (1.0 - 2.0 * ((x >> i) & 1))) for i in range(nout)])
    np.savez_compressed(PLAIN_LARGE, idx=idx, amp=psi[idx], probs=probs, z=z,
                        norm=np.array(np.sqrt(np.sum(p2))), seconds=np.array(wall),
                        threads=np.array(threads), commands=np.array(len(wl.pattern.cmds)),
                        cpu=np.array(_cpu_model()))
    print(f"plain_large: {len(wl.pattern.cmds)} commands in {wall:.1f} s on {threads} threads -> {PLAIN_LARGE}")


def gradient(sets=(0, 1)) -> None:
    wl, alphas = W.ansatz()
    threads = os.cpu_count() or 1
    oc.set_threads(1)  # one oracle per worker thread
    out = {}
    t0 = time.perf_counter()
    for b in sets:
        a = alphas[b]
        n = a.size

        def shift(k):
            oc.set_threads(1)  # the OpenMP thread count is per calling thread
            return float(oc.param_shift_grad(wl.pattern, wl.outcomes, a, indices=[k])[k])

        with ThreadPoolExecutor(threads) as ex:
            g = np.array(list(ex.map(shift, range(n))))
        out[f"grad{b}"] = g
        out[f"loss{b}"] = np.array(oc.loss_at(wl.pattern, wl.outcomes, a))
        print(f"gradient: set {b} done ({time.perf_counter() - t0:.1f} s)", flush=True)
    np.savez_compressed(GRADIENT, sets=np.array(sets), seconds=np.array(time.perf_counter() - t0),
                        threads=np.array(threads), **out)
    print(f"gradient -> {GRADIENT}")


if __name__ == "__main__":
    what = sys.argv[1:] or ["plain_large", "gradient"]
    for w in what:
        {"plain_large": plain_large, "gradient": gradient}[w]()
