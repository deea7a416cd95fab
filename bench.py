#!/usr/bin/env python3
"""Benchmark of 1WQC pattern execution on one MI355X.

Workload (the large plain configuration): a random circuit on 24 logical
qubits of 2000 J(alpha) gates (alpha uniform in [0, 2pi)) and 300 CZ gates on
random pairs, translated into a measurement pattern (J(alpha) = N w; E u w;
M u^(-alpha); X w^(s_u), CZ = E) with live width 24 <-> 25 (2^25 complex64
amplitudes, 256 MiB), seeded forced outcomes and a normalised complex Gaussian
input state already resident in device memory.

One step = one whole run of the pattern (every N, E, M, X command as HIP
kernels, FP64 probability reductions) plus the read-out of the 2^24 output
amplitudes into a device buffer.

Printed: one JSON line with the metric (non-trivial pattern commands per
second), the roofline of the dominant kernel (HIP events around every launch
of one extra profiled step), a measured device-copy ceiling, the fused
executor's figures and the other workloads' legs, and the FP64 oracle timed
on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = dict(n_logical=24, n_j=2000, n_cz=300)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(name: str) -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1604_05659_amd", "csrc", name), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM-side bytes per launch from the committed rocprofv3 counter summary
    (profiles/traffic.json), or None when it is missing or was taken on a
    different version of the kernel's source file."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    e = d.get(kernel)
    if not e or e.get("source_hash") != source_hash(e.get("source", "owqs_kernels.hip")):
        return None
    return e.get("bytes_per_launch")


def kernel_table(prof):
    return {k: {"launches": v["launches"], "avg_us": round(1e3 * v["ms"] / v["launches"], 2),
                "GB/s": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1)} for k, v in prof.items()}


def time_exec(owqs, torch, pat, inp, out, exec_, steps, warmup, profile=True):
    pat.set_exec(exec_)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        pat.run(inp)
        pat.read_state(out, check=False)
    if warmup:
        pat.check()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        pat.run(inp)
        pat.read_state(out, check=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pat.check()
    ev_ms = ev0.elapsed_time(ev1)
    prof = pat.run_profiled(inp) if profile else None
    return wall, ev_ms, prof


def roofline_of(prof, kernel_names):
    dom = max(prof, key=lambda k: prof[k]["ms"])
    e = prof[dom]
    avg_s = e["ms"] / e["launches"] / 1e3
    per_launch = e["bytes"] / e["launches"]
    achieved = per_launch / avg_s / 1e9
    tr = measured_traffic(kernel_names.get(dom, dom))
    return dom, {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": tr,
        "kernel": dom,
        "bytes_per_launch": per_launch,
        "avg_launch_us": round(avg_s * 1e6, 2),
        "launches_per_step": e["launches"],
    }


def cpu_baseline(wl_gates, psi_in, seconds_hint):
    """Oracle (complex128, OpenMP over all host cores) on the first gates of
    the same circuit at the same width; returns the JSON object."""
    import owqs_workloads as W
    from oracle import core as oc

    threads = os.cpu_count() or 1
    threads = oc.set_threads(threads)
    n_gates = 12
    gates = wl_gates[:n_gates]
    pat = W.circuit_to_pattern(WORKLOAD["n_logical"], gates, prepare_zero=False)
    outc = W.outcome_bits(pat.n_meas(), W.rng(2, W.P_OUTCOME, 0))
    x = psi_in.astype(np.complex128)
    t0 = time.perf_counter()
    oc.run(pat, outc, x, oc.MODE_OWQS)
    dt = time.perf_counter() - t0
    nt = pat.nontrivial_count(outc)
    # one thread, on the first two gates
    g1 = wl_gates[:2]
    pat1 = W.circuit_to_pattern(WORKLOAD["n_logical"], g1, prepare_zero=False)
    out1 = W.outcome_bits(pat1.n_meas(), W.rng(2, W.P_OUTCOME, 0))
    oc.set_threads(1)
    t0 = time.perf_counter()
    oc.run(pat1, out1, x, oc.MODE_OWQS)
    dt1 = time.perf_counter() - t0
    oc.set_threads(threads)
    nt1 = pat1.nontrivial_count(out1)
    res = {
        "value": round(nt / dt, 3),
        "unit": "commands/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"first {n_gates} gates ({len(pat.cmds)} commands, {nt} non-trivial) of the same circuit "
                   f"at live width 24<->25, complex128, {dt:.1f} s wall"),
        "nproc": os.cpu_count(),
        "cpu_model": _cpu_model(),
        "one_thread": {"value": round(nt1 / dt1, 3), "unit": "commands/s", "cores": 1,
                       "sample": f"first 2 gates ({len(pat1.cmds)} commands, {nt1} non-trivial), {dt1:.1f} s wall"},
    }
    # the whole pattern, timed when the oracle wrote the stored expected values
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "plain_large_full.npz")
    if os.path.exists(gold):
        g = np.load(gold, allow_pickle=False)
        res["whole_pattern"] = {"seconds": round(float(g["seconds"]), 1), "threads": int(g["threads"]),
                                "cpu_model": str(g["cpu"]), "commands": int(g["commands"]),
                                "value": round(nt_all_of(wl_gates) / float(g["seconds"]), 3),
                                "unit": "commands/s",
                                "where": "the build container (not the GPU host), tests/golden/make_goldens.py"}
    return res


def nt_all_of(wl_gates):
    """Non-trivial commands of the whole large pattern with its seeded outcomes."""
    import owqs_workloads as W
    pat = W.circuit_to_pattern(WORKLOAD["n_logical"], wl_gates, prepare_zero=False)
    return pat.nontrivial_count(W.outcome_bits(pat.n_meas(), W.rng(2, W.P_OUTCOME, 0)))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def bench_batched(owqs, torch, W, ctx, steps):
    """512 random J/CZ patterns (live widths 8..20, 50..800 commands each):
    one owqs_run_batch call (one captured graph) versus the same plans run
    one pattern after another, and versus the plain executor one pattern
    after another."""
    wls = [W.batched_random(i) for i in range(512)]
    pats, ins, outs = [], [], []
    for wl in wls:
        p = owqs.Pattern(ctx, wl.pattern)
        p.set_mode(owqs.MODE_OWQS)
        p.set_outcomes(wl.outcomes)
        pats.append(p)
        ins.append(torch.as_tensor(wl.input_state).cuda())
        outs.append(torch.empty(1 << len(wl.pattern.outputs), dtype=torch.complex64, device="cuda"))
    n_cmds = sum(len(wl.pattern.cmds) for wl in wls)
    widths = [p.plan_info()[0] for p in pats]
    # batched: the tile size of the wide plans picked for the batch
    tile_bits, _ = owqs.tune_batch(ctx, pats, ins, outs)
    owqs.run_batch(ctx, pats, ins, outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        owqs.run_batch(ctx, pats, ins, outs)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    for p in pats:
        p.check()
    batched_out = [o.clone() for o in outs]
    # the same plans (default executor, captured graphs), one pattern after another
    for p, x, o in zip(pats, ins, outs):
        p.run(x)
        p.read_state(o, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, x, o in zip(pats, ins, outs):
        p.run(x)
        p.read_state(o, check=False)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    # plain, one pattern after another
    for p in pats:
        p.set_exec(owqs.EXEC_PLAIN)
        p.set_graph(False)
    for p, x, o in zip(pats[:8], ins, outs):
        p.run(x)
        p.read_state(o, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, x, o in zip(pats, ins, outs):
        p.run(x)
        p.read_state(o, check=False)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    diff = max(float((a - b).abs().max().item()) for a, b in zip(batched_out, outs))
    for p in pats:
        p.close()
    return {
        "workload": "512 random J/CZ patterns, live width 8..20, 50..800 commands, Gaussian inputs, OWQS",
        "patterns": len(pats),
        "commands": n_cmds,
        "lds_resident": int(sum(w <= 14 for w in widths)),
        "tile_bits": tile_bits,
        "batched_patterns_per_s": round(len(pats) / t_batch, 1),
        "batched_ms": round(1e3 * t_batch, 3),
        "sequential_patterns_per_s": round(len(pats) / t_seq, 1),
        "sequential_ms": round(1e3 * t_seq, 3),
        "sequential_note": "the same plans (default executor, graphs on) run one pattern after another",
        "speedup_vs_sequential": round(t_seq / t_batch, 2),
        "plain_patterns_per_s": round(len(pats) / t_plain, 1),
        "plain_ms": round(1e3 * t_plain, 3),
        "plain_note": "plain executor (one kernel per command, no graph), one pattern after another",
        "speedup": round(t_plain / t_batch, 2),
        "max_abs_diff_batched_vs_plain": diff,
    }


def bench_recognition(owqs, torch, W, ctx, steps):
    """Recognition problem: a 12-input J/CZ pattern (300 J, 60 CZ) on all 4096
    basis inputs in one LDS-resident launch, versus the plain executor on a
    sample of 64 inputs."""
    wl = W.recognition()
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_EOWQS)
    p.set_outcomes(wl.outcomes)
    out = p.run_basis()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p.run_basis(out=out)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / steps
    p.check()
    p.set_exec(owqs.EXEC_PLAIN)
    x = torch.zeros(4096, dtype=torch.complex64, device="cuda")
    col = torch.empty(1 << 12, dtype=torch.complex64, device="cuda")
    n_sample = 64
    x[0] = 1
    p.run(x)
    p.read_state(col)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_sample):
        x.zero_()
        x[k] = 1
        p.run(x)
        p.read_state(col, check=False)
    torch.cuda.synchronize()
    t_p = (time.perf_counter() - t0) / n_sample
    diff = float((col - out[n_sample - 1]).abs().max().item())
    w = p.plan_info()[0]
    p.close()
    return {
        "workload": "recognition: 12 inputs, 300 J + 60 CZ (1260 commands), all 4096 basis inputs, EOWQS",
        "inputs": 4096,
        "plan_width": w,
        "batched_inputs_per_s": round(4096 / t_b, 1),
        "batched_ms": round(1e3 * t_b, 3),
        "plain_inputs_per_s": round(1 / t_p, 1),
        "speedup": round(t_p * 4096 / t_b, 1),
        "max_abs_diff_vs_plain": diff,
    }


def bench_adjoint(owqs, torch, W, ctx, steps):
    """Differentiated workload: 16-qubit layered ansatz, 25 layers, 400 M
    angles, 64 angle sets; one owqs_adjoint call = forward + checkpointed
    backward for all sets."""
    wl, sets = W.ansatz()
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_EOWQS)
    p.set_outcomes(wl.outcomes)
    p.adjoint(sets)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        loss, grad = p.adjoint(sets)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    w = p.plan_info()[0]
    p.close()
    return {
        "workload": "layered ansatz, 16 qubits, 25 layers (400 angles), 64 angle sets, loss sum_i <Z_i>, EOWQS",
        "sets": int(sets.shape[0]),
        "angles": int(sets.shape[1]),
        "plan_width": w,
        "ms_forward_backward": round(1e3 * t, 3),
        "sets_per_s": round(sets.shape[0] / t, 1),
        "gradient_entries_per_s": round(sets.size / t, 1),
    }


def bench_cluster(owqs, torch, W, ctx, steps):
    """20 x 200 cluster measured column by column (width 21), OWQS."""
    wl = W.cluster()
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_OWQS)
    p.set_outcomes(wl.outcomes)
    out = torch.empty(1 << 20, dtype=torch.complex64, device="cuda")
    nt = wl.pattern.nontrivial_count(wl.outcomes)
    res = {"workload": "2D cluster 20 x 200, angles k pi/4, live width 21, OWQS",
           "commands_listed": len(wl.pattern.cmds), "commands_nontrivial": nt}
    for name, ex in (("plain", owqs.EXEC_PLAIN), ("fused", owqs.EXEC_FUSED)):
        p.set_exec(ex)
        p.run(None)
        p.read_state(out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            p.run(None)
            p.read_state(out, check=False)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        p.check()
        res[name] = {"ms_per_run": round(1e3 * t, 3), "commands_per_s": round(nt / t, 1),
                     "plan_steps": p.plan_info()[1], "passes": p.plan_info()[2]}
    t0 = time.perf_counter()
    ok, first = p.certify()
    t_cert = time.perf_counter() - t0
    t0 = time.perf_counter()
    ex, depth, _ = p.gflow()
    t_gf = time.perf_counter() - t0
    res["eowqs_certificate"] = {"all_certified": bool(ok.all()), "host_ms": round(1e3 * t_cert, 1),
                                "gflow_exists": ex, "gflow_depth": depth, "gflow_host_ms": round(1e3 * t_gf, 1)}
    p.close()
    res["proa"] = bench_proa(owqs, torch, W, ctx, wl, steps)
    return res


def bench_proa(owqs, torch, W, ctx, wl, steps):
    """The same cluster as a standard-form pattern (all N, all E, then the
    M's: 4000 qubits live at once), reordered on the host by the library
    (PROA, Sec. 4.3) and run fused; compared with the column-by-column order."""
    std = W.standard_form(wl.pattern)
    src = owqs.Pattern(ctx, std)
    t0 = time.perf_counter()
    re, stats = src.reorder()
    host_ms = 1e3 * (time.perf_counter() - t0)
    spec = re.commands()
    per_q = dict(zip([c[1] for c in wl.pattern.cmds if c[0] == "M"], (int(b) for b in wl.outcomes)))
    re.set_mode(owqs.MODE_OWQS)
    re.set_exec(owqs.EXEC_FUSED)
    re.set_outcomes(np.array([per_q[c[1]] for c in spec.cmds if c[0] == "M"], np.uint8))
    out = torch.empty(1 << 20, dtype=torch.complex64, device="cuda")
    re.run(None)
    re.read_state(out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        re.run(None)
        re.read_state(out, check=False)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    re.check()
    col = owqs.Pattern(ctx, wl.pattern)
    col.set_outcomes(wl.outcomes)
    col.set_exec(owqs.EXEC_FUSED)
    col.run(None)
    ref = col.read_state()
    diff = float((ref - out).abs().max().item())
    col.close()
    res = {"source_live_width": src.max_live, "host_reorder_ms": round(host_ms, 1),
           "max_state_space": stats["max_state_space"], "live_width": stats["max_live"], "alpha": stats["alpha"],
           "fused_ms_per_run": round(1e3 * t, 3), "max_abs_diff_vs_column_order": diff}
    re.close()
    src.close()
    return res


def bench_substates(owqs, torch, W, ctx, steps):
    """Sub-state executor (Sec. 4.1): (1) three 16-qubit circuits side by side
    (48 inputs and outputs, one vector would need 2^51 amplitudes), input as
    three factors; (2) two 13-qubit circuits merged by one E at the end: a
    2^13 x 2^13 tensor product (k_kron) timed with events."""
    g = np.random.default_rng([160405659, 9, 0])
    parts = [W.circuit_to_pattern(16, W.random_jcz_circuit(16, 400, 60, g)) for _ in range(3)]
    pat_def = W.disjoint_union(parts)
    outc = g.integers(0, 2, pat_def.n_meas()).astype(np.uint8)
    ins = [torch.as_tensor(W.gaussian_state(16, g)).cuda() for _ in parts]
    p = owqs.Pattern(ctx, pat_def)
    p.set_exec(owqs.EXEC_SUBSTATES)
    p.set_outcomes(outc)
    p.run_factors(ins)
    p.read_substates()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p.run_factors(ins)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    p.check()
    nt = pat_def.nontrivial_count(outc)
    res = {"components": {
        "workload": "3 random J/CZ circuits of 16 logical qubits (400 J + 60 CZ each) side by side, "
                    "inputs as 3 factors, OWQS",
        "single_vector_live_width": pat_def.max_live(), "widest_substate": p.plan_info()[0],
        "commands_nontrivial": nt, "ms_per_run": round(1e3 * t, 3), "commands_per_s": round(nt / t, 1)}}
    p.close()
    # one large merge: two 13-qubit path graph states (N and E only: each
    # grows by prepares, no merge), then one E across them, a 2^13 x 2^13
    # tensor product; no measurement
    na = 13
    cmds = []
    for base in (0, 100):
        for k in range(na):
            cmds.append(("N", base + k))
            if k:
                cmds.append(("E", base + k - 1, base + k))
    cmds.append(("E", 0, 100))
    pat_def = W.Pattern([], [k for k in range(na)] + [100 + k for k in range(na)], cmds)
    outc = np.zeros(0, np.uint8)
    p = owqs.Pattern(ctx, pat_def)
    p.set_exec(owqs.EXEC_SUBSTATES)
    p.set_outcomes(outc)
    p.run(None)
    kr_ms, kr_bytes, n = 0.0, 0.0, 0
    for _ in range(max(steps, 3)):
        k = p.run_profiled(None).get("kron(merge)", {"ms": 0.0, "bytes": 0.0, "launches": 0})
        kr_ms += k["ms"]
        kr_bytes += k["bytes"]
        n += k["launches"]
    p.check()
    avg_us = 1e3 * kr_ms / max(n, 1)
    gbs = kr_bytes / max(kr_ms, 1e-12) / 1e6
    res["merge"] = {"workload": f"two {na}-qubit path graph states, then one E across them: "
                                f"a 2^{na} x 2^{na} tensor product (2^{2 * na} amplitudes written)",
                    "kron_launches": n, "kron_avg_us": round(avg_us, 2),
                    "kron_bytes_per_launch": kr_bytes / max(n, 1),
                    "kron_GBs": round(gbs, 1), "kron_frac_of_8TBs": round(gbs / 8000.0, 4)}
    p.close()
    return res


def bench_widths(owqs, torch, W, ctx):
    """The plain kernels at live widths 24..28 (128 MiB .. 2 GiB of complex64):
    at 2^24 and 2^25 the vector is close to the 256 MB Infinity Cache, so
    wider runs show the HBM-only rate.  A short random J/CZ circuit per
    width, profiled with events (element-level algorithmic bytes)."""
    out = {}
    for nl in (23, 24, 25, 26, 27):
        g = np.random.default_rng([160405659, 10, 0, nl])
        pat_def = W.circuit_to_pattern(nl, W.random_jcz_circuit(nl, 12, 4, g))
        outc = g.integers(0, 2, pat_def.n_meas()).astype(np.uint8)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(nl)
        re = torch.randn(1 << nl, device="cuda", generator=gen, dtype=torch.float32)
        im = torch.randn(1 << nl, device="cuda", generator=gen, dtype=torch.float32)
        inp = torch.complex(re, im)
        inp /= torch.linalg.vector_norm(inp)
        del re, im
        p = owqs.Pattern(ctx, pat_def)
        p.set_exec(owqs.EXEC_PLAIN)
        p.set_outcomes(outc)
        p.run(inp)
        p.check()
        prof = p.run_profiled(inp)
        p.check()
        row = {}
        for k, name in (("measure(M)", "M"), ("prepare(N)", "N"), ("pauli_x(X)", "X"), ("cz(E)", "E")):
            v = prof.get(k)
            if v:
                gbs = v["bytes"] / (v["ms"] / 1e3) / 1e9
                row[name] = {"avg_us": round(1e3 * v["ms"] / v["launches"], 2), "GB/s": round(gbs, 1),
                             "frac": round(gbs / 8000.0, 3)}
        out[f"2^{nl + 1}"] = row
        p.close()
        del inp
        torch.cuda.empty_cache()
    return out


def bench_sampled(owqs, torch, pat, inp, out, n_nontriv, steps, warmup):
    """The same large pattern with its outcomes drawn on the device from seeded
    uniforms (plain plan, signals resolved on the GPU, replayed as a graph).
    The pattern is deterministic, so the output must equal the forced run's."""
    pat.set_exec(owqs.EXEC_PLAIN)
    pat.run(inp)
    pat.read_state(out)
    forced = out.clone()
    u = np.random.default_rng([160405659, 2, 4, 0]).random(pat.n_meas)
    pat.set_uniforms(u)
    for _ in range(warmup):
        pat.run(inp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pat.run(inp)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    pat.read_state(out)
    drawn = pat.read_outcomes()
    res = {"workload": "plain_large with outcomes drawn on the device (u <= p_0 gives 0; seeded uniforms), "
                       "plain plan: every window drawn by one thread (p = 1/2), every other step one kernel",
           "ms_per_run": round(1e3 * dt, 3), "commands_per_s": round(n_nontriv / dt, 1),
           "ones_drawn": int(drawn.sum()), "max_abs_diff_vs_forced": float((out - forced).abs().max().item())}
    # the fused plan: every M is a window with p = 1/2, so the outcomes follow
    # from the uniforms and the tile passes run with per-run coefficient tables
    pat.set_exec(owqs.EXEC_FUSED)
    for _ in range(warmup):
        pat.run(inp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pat.run(inp)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    pat.read_state(out)
    same = bool((pat.read_outcomes() == drawn).all())
    res["fused"] = {"ms_per_run": round(1e3 * dt, 3), "commands_per_s": round(n_nontriv / dt, 1),
                    "same_outcomes_as_plain": same,
                    "max_abs_diff_vs_forced": float((out - forced).abs().max().item())}
    pat.set_uniforms(None)
    pat.set_exec(owqs.EXEC_PLAIN)
    return res


def copy_ceiling(torch):
    """A measured copy ceiling next to the 8 TB/s peak: torch's device copy
    of 2^25 complex64 (256 MiB, about the size of the Infinity Cache) and of
    2^28 (2 GiB, beyond it), event-timed; bytes = read + write."""
    out = {}
    for n in (25, 28):
        a = torch.empty(1 << n, dtype=torch.complex64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"2^{n}"] = {"us": round(1e3 * ms, 2), "GB/s": round(2 * a.numel() * 8 / (ms / 1e3) / 1e9, 1)}
        del a, b
    return out


def bench_small(owqs, torch, W, ctx, steps):
    """The small plain pattern (4 logical qubits, 106 commands): latency of
    one run plus read-out through the C ABI, host calls included (the default
    executor runs a pattern this narrow in one workgroup's LDS)."""
    wl = W.plain_small()
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_OWQS)
    p.set_outcomes(wl.outcomes)
    out = torch.empty(16, dtype=torch.complex64, device="cuda")
    p.run(None)
    p.read_state(out)
    reps = 200 * steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        p.run(None)
        p.read_state(out, check=False)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    p.close()
    return {"workload": "plain_small: 4 logical qubits, 20 J + 6 CZ, 106 commands, OWQS, one workgroup in LDS "
                        "(default executor), run + read-out through the Python binding",
            "us_per_pattern": round(1e6 * t, 2)}


def pmc_probe():
    """The first 8 gates of the large circuit at its full width (24 <-> 25),
    run once with the plain executor and once fused, each command its own
    dispatch (no graph): a few dozen dispatches of exactly the kernels and
    launch shapes of the timed workload, for hardware-counter passes."""
    import torch
    import owqs_workloads as W
    import paper_1604_05659_amd as owqs

    wl = W.plain_large(**WORKLOAD)
    gates = wl.meta["gates"][:8]
    pat_def = W.circuit_to_pattern(WORKLOAD["n_logical"], gates)
    outc = W.outcome_bits(pat_def.n_meas(), np.random.default_rng(1))
    ctx = owqs.Context(0)
    p = owqs.Pattern(ctx, pat_def)
    p.set_mode(owqs.MODE_OWQS)
    p.set_outcomes(outc)
    p.set_graph(False)
    inp = torch.as_tensor(wl.input_state).cuda()
    out = torch.empty(1 << 24, dtype=torch.complex64, device="cuda")
    for ex in (owqs.EXEC_PLAIN, owqs.EXEC_FUSED):
        p.set_exec(ex)
        p.run(inp)
        p.read_state(out)
    torch.cuda.synchronize()
    p.close()
    print(json.dumps({"pmc_probe": "done", "commands": len(pat_def.cmds), "counts": pat_def.counts()}), flush=True)


def tile_probe():
    """One fused run of the large workload (OWQS, tile bits 12) after one
    warm-up run: the dispatches hardware-counter passes over k_tile read."""
    import torch
    import owqs_workloads as W
    import paper_1604_05659_amd as owqs
    wl = W.plain_large(**WORKLOAD)
    ctx = owqs.Context(0)
    p = owqs.Pattern(ctx, wl.pattern)
    p.set_mode(owqs.MODE_OWQS)
    p.set_outcomes(wl.outcomes)
    p.set_exec(owqs.EXEC_FUSED)
    p.set_tile_bits(12)
    inp = torch.as_tensor(wl.input_state).cuda()
    p.run(inp)
    torch.cuda.synchronize()
    log(f"[bench] tile probe: plan {p.plan_info()}")
    p.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fused", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-sampled", action="store_true")
    ap.add_argument("--no-substates", action="store_true")
    ap.add_argument("--no-widths", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the extra event-timed step (for counter collection runs)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="one short run at full width, few dispatches: for rocprofv3 --pmc passes")
    ap.add_argument("--batch-probe", action="store_true",
                    help="only the batched leg (512 patterns, one graph per call, 3 calls after a warm-up): for "
                         "rocprofv3 kernel traces of the batch")
    ap.add_argument("--tile-probe", action="store_true",
                    help="one fused run of the large workload at tile bits 12 (22 tile passes): for rocprofv3 "
                         "--pmc passes over the tile kernel")
    ap.add_argument("--only-plain", action="store_true",
                    help="run only the plain executor on the large workload (for counter collection runs)")
    args = ap.parse_args()
    if args.pmc_probe:
        pmc_probe()
        return
    if args.tile_probe:
        tile_probe()
        return
    if args.batch_probe:
        import torch
        import owqs_workloads as W
        import paper_1604_05659_amd as owqs
        ctx = owqs.Context(0)
        print(json.dumps({"batch_probe": bench_batched(owqs, torch, W, ctx, 3)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs a pattern on a single MI355X "
              "(no multi-GPU path); use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.only_plain:
        args.no_fused = args.no_batch = args.no_adjoint = args.no_sampled = args.no_cpu_baseline = True
        args.no_substates = True
        args.no_widths = True

    import torch
    import owqs_workloads as W
    import paper_1604_05659_amd as owqs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    log("[bench] generating workload")
    wl = W.plain_large(**WORKLOAD)
    pat_def = wl.pattern
    counts = pat_def.counts()
    n_all = len(pat_def.cmds)
    n_nontriv = pat_def.nontrivial_count(wl.outcomes)

    ctx = owqs.Context(0)
    pat = owqs.Pattern(ctx, pat_def)
    pat.set_mode(owqs.MODE_OWQS)
    pat.set_outcomes(wl.outcomes)
    inp = torch.as_tensor(wl.input_state).cuda()
    out = torch.empty(1 << len(pat_def.outputs), dtype=torch.complex64, device="cuda")
    names = {"measure(M)": "k_measure", "prepare(N)": "k_prepare", "cz(E)": "k_cz", "pauli_x(X)": "k_x",
             "jwindow(NEMX)": "k_jwindow", "tile(group)": "k_tile"}

    log("[bench] plain executor")
    wall, ev_ms, prof = time_exec(owqs, torch, pat, inp, out, owqs.EXEC_PLAIN, args.steps, args.warmup,
                                  not args.no_profile)
    probs = pat.read_probs()
    ms_step = 1e3 * wall / args.steps
    result = {
        "metric": "pattern commands/s & HBM GB/s at 2^25 amps; batched vs plain at err<=1e-5",
        "value": round(n_nontriv / (ms_step / 1e3), 1),
        "unit": "commands/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("plain_large: random J/CZ circuit on 24 logical qubits, 2000 J(alpha) + 300 CZ, "
                         "pattern of 8300 commands, live width 24<->25 (2^25 complex64 amplitudes), "
                         "complex Gaussian input, seeded forced outcomes, OWQS mode (FP64 probabilities)"),
            "exec": "plain (one kernel per non-trivial command, replayed as a HIP graph)",
            "commands_listed": n_all,
            "commands_nontrivial": n_nontriv,
            "counts": counts,
        },
        "commands_all_per_s": round(n_all / (ms_step / 1e3), 1),
        "event_ms_per_step": round(ev_ms / args.steps, 3),
        "checks": {"max_abs_p_minus_half": float(np.max(np.abs(probs - 0.5)))},
    }
    if prof:
        _, roof = roofline_of(prof, names)
        step_bytes = sum(v["bytes"] for v in prof.values())
        result["hbm_gbs_step"] = round(step_bytes / (ms_step / 1e3) / 1e9, 1)
        result["roofline"] = roof
        result["kernels"] = kernel_table(prof)

    result["copy_ceiling"] = copy_ceiling(torch)

    if not args.no_fused:
        log("[bench] fused executor (tile size picked by the autotuner)")
        pat.set_exec(owqs.EXEC_FUSED)
        tile_bits, _ = pat.tune(inp)
        wall_f, ev_f, prof_f = time_exec(owqs, torch, pat, inp, out, owqs.EXEC_FUSED, args.steps, args.warmup,
                                         not args.no_profile)
        probs_f = pat.read_probs()
        fused_passes = pat.plan_info()[2]
        fused_out = out.clone()
        pat.set_exec(owqs.EXEC_PLAIN)
        pat.run(inp)
        pat.read_state(out)
        diff = float((fused_out - out).abs().max().item())
        ms_f = 1e3 * wall_f / args.steps
        result["fused"] = {
            "value": round(n_nontriv / (ms_f / 1e3), 1),
            "unit": "commands/s",
            "ms_per_step": round(ms_f, 3),
            "live_width": 24,
            "tile_bits": tile_bits,
            "passes": fused_passes,
            "max_abs_diff_vs_plain": diff,
            "max_abs_p_minus_half": float(np.max(np.abs(probs_f - 0.5))),
            "probability_work": ("OWQS with windows of p = 1/2 recorded without sums (reading G24: a window whose "
                                 "new qubit meets the measured one through an odd number of E has p = 1/2 exactly; "
                                 "the tile pass that ends a run of up to 128 such windows sums the norm of its "
                                 "output and renormalises)"),
        }
        # the same plan with every probability summed (the paper's OWQS work per M)
        pat.set_sum_all(True)
        pat.set_exec(owqs.EXEC_FUSED)
        pat.set_tile_bits(tile_bits)
        wall_s, _, _ = time_exec(owqs, torch, pat, inp, out, owqs.EXEC_FUSED, args.steps, args.warmup, False)
        probs_s = pat.read_probs()
        diff_s = float((out - fused_out).abs().max().item())
        ms_s = 1e3 * wall_s / args.steps
        result["fused"]["sum_every_m"] = {
            "value": round(n_nontriv / (ms_s / 1e3), 1),
            "unit": "commands/s",
            "ms_per_step": round(ms_s, 3),
            "passes": pat.plan_info()[2],
            "max_abs_diff_vs_default_fused": diff_s,
            "max_abs_p_minus_half": float(np.max(np.abs(probs_s - 0.5))),
            "probability_work": "OWQS with every window's probability summed in FP64 (owqs_set_sum_all)",
        }
        pat.set_sum_all(False)
        if prof_f:
            _, roof_f = roofline_of(prof_f, names)
            result["fused"]["roofline"] = roof_f
            result["fused"]["kernels"] = kernel_table(prof_f)
            # the tile pass against the vector ALU, on the FP32 work it runs: a
            # window applied alone is 8 FP32 operations per amplitude pair (4
            # lane operations per amplitude), a composed 2x2 map 16 (8); on the
            # live width the passes run at; the peak is 256 CUs x 64 FP32 lanes
            # x 2.4 GHz (packed FP32 is not used)
            tile_us = roof_f.get("avg_launch_us", 0.0) * roof_f.get("launches_per_step", 0)
            tw, tm, tc = pat.plan_tile_work()
            result["fused"]["composition"] = {
                "windows_alone": tw, "maps": tm, "windows_in_maps": tc,
                "note": "windows in a row on one register-round position, with no E / Z on its bit between them, "
                        "run as one 2x2 map (FP64 product rounded to FP32)"}
            if tile_us > 0:
                lane_ops = float(1 << 24) * (4.0 * tw + 8.0 * tm)
                achieved = lane_ops / (tile_us * 1e-6) / 1e12
                peak = 256 * 64 * 2.4e9 / 1e12
                per_window = 4.0 * float(1 << 24) * counts["M"] / (tile_us * 1e-6) / 1e12
                result["fused"]["alu_roofline"] = {
                    "bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2),
                    "unit": "Tlane-op/s", "frac": round(achieved / peak, 4),
                    "work": "executed FP32 work at 2^24 amplitudes: 4 lane operations per amplitude for each of the "
                            "%d windows applied alone, 8 for each of the %d composed maps (E / Z, set-up and LDS "
                            "rounds not counted), over the tile passes' event time" % (tw, tm),
                    "per_window_equivalent": {
                        "achieved": round(per_window, 2), "frac": round(per_window / peak, 4),
                        "work": "4 lane operations per amplitude for every one of the %d windows, as if none "
                                "were composed, over the same time" % counts["M"]}}
        if prof:
            # each tile pass carries about nontrivial / passes commands in one
            # HBM round trip: the plain executor's algorithmic bytes for the
            # same result, over the fused run time
            result["fused"]["commands_per_pass"] = round(n_nontriv / max(fused_passes, 1), 1)
            result["fused"]["bound_note"] = ("a tile pass applies all its steps between one HBM read and write of the "
                                             "vector; its time is the steps' VALU work and LDS rounds, so the HBM "
                                             "fraction of a pass is not its limit")
            result["fused"]["plain_equivalent_GBs"] = round(step_bytes / (ms_f / 1e3) / 1e9, 1)
    if not args.no_sampled:
        log("[bench] drawn outcomes")
        result["sampled"] = bench_sampled(owqs, torch, pat, inp, out, n_nontriv, args.steps, args.warmup)
    pat.close()

    if not args.no_batch:
        log("[bench] batched workload")
        result["batched"] = bench_batched(owqs, torch, W, ctx, args.steps)
        log("[bench] recognition workload")
        result["recognition"] = bench_recognition(owqs, torch, W, ctx, args.steps)
        log("[bench] cluster workload")
        result["cluster"] = bench_cluster(owqs, torch, W, ctx, args.steps)
        log("[bench] small workload")
        result["small"] = bench_small(owqs, torch, W, ctx, args.steps)
    if not args.no_widths:
        log("[bench] plain kernels at widths 24..28")
        result["widths"] = bench_widths(owqs, torch, W, ctx)
        if "roofline" in result:
            # above the 256 MB Infinity Cache the vector streams from HBM only
            result["roofline"]["above_cache"] = {
                w: {k: v["frac"] for k, v in row.items()} for w, row in result["widths"].items()
                if w in ("2^26", "2^27", "2^28")}
    if not args.no_substates:
        log("[bench] sub-state executor")
        result["substates"] = bench_substates(owqs, torch, W, ctx, args.steps)
    if not args.no_adjoint:
        log("[bench] differentiated workload")
        result["adjoint"] = bench_adjoint(owqs, torch, W, ctx, args.steps)

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(wl.meta["gates"], wl.input_state, 20)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
