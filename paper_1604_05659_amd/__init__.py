"""Python binding of libowqs: 1WQC pattern execution on an MI355X (gfx950).

Argument marshalling only: every step of a run executes in the HIP kernels of
``libowqs.so`` (see ``include/owqs.h``).  PyTorch supplies device memory and
the current stream.  Importing this package fails loudly when the library has
not been built; there is no CPU fallback.

Typical use::

    import paper_1604_05659_amd as owqs
    ctx = owqs.Context(0)
    pat = owqs.Pattern(ctx, pattern)          # pattern: .inputs/.outputs/.cmds
    pat.set_outcomes(bits)
    pat.run(psi_in)                           # complex64 CUDA tensor
    psi_out = pat.read_state()                # complex64 CUDA tensor
"""
from __future__ import annotations

import collections
import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libowqs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python paper_1604_05659_amd/build.py` "
        "(or __graft_entry__.build()) first. There is no CPU fallback.")

# PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Import it first
# so that libowqs binds to that same runtime instead of loading a second copy
# from /opt/rocm: device pointers and streams are then shared with torch.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

OK = 0
E_INVALID_ARG, E_PATTERN, E_ZERO_PROB, E_WIDTH, E_NOMEM, E_HIP, E_NOT_DETERMINISTIC, E_STATE = range(-1, -9, -1)
MODE_OWQS, MODE_EOWQS, MODE_EOWQS_CHECK = 0, 1, 2
EXEC_PLAIN, EXEC_FUSED, EXEC_AUTO, EXEC_SUBSTATES = 0, 1, 2, 3
OPS = {"N": 0, "E": 1, "M": 2, "X": 3, "Z": 4}
KINDS = {0: "prepare(N)", 1: "cz(E)", 2: "measure(M)", 3: "pauli_x(X)", 4: "pauli_z(Z)", 5: "jwindow(NEMX)",
         6: "finish(FP64)", 7: "tile(group)", 8: "kron(merge)"}
NUM_KINDS = 9


class OwqsCmd(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("s_off", ctypes.c_int32), ("s_len", ctypes.c_int32),
                ("t_off", ctypes.c_int32), ("t_len", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("angle", ctypes.c_double)]


assert ctypes.sizeof(OwqsCmd) == 40

_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
MAX_WIDTH = 34  # OWQS_MAX_WIDTH
NOALLOC_MAX_WIDTH = 22  # OWQS_NOALLOC_MAX_WIDTH
_sig = {
    "owqs_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "owqs_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp)]),
    "owqs_ctx_destroy": (None, [_vp]),
    "owqs_last_error": (ctypes.c_char_p, [_vp]),
    "owqs_pattern_create": (ctypes.c_int, [_vp, ctypes.POINTER(OwqsCmd), ctypes.c_size_t, _i32p,
                                           ctypes.c_size_t, _i32p, ctypes.c_int32, _i32p, ctypes.c_int32,
                                           ctypes.POINTER(_vp)]),
    "owqs_pattern_from_text": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "owqs_pattern_destroy": (None, [_vp]),
    "owqs_pattern_info": (ctypes.c_int, [_vp, _i32p, _i32p, _i32p, _i32p, ctypes.POINTER(ctypes.c_size_t)]),
    "owqs_set_mode": (ctypes.c_int, [_vp, ctypes.c_int]),
    "owqs_set_exec": (ctypes.c_int, [_vp, ctypes.c_int]),
    "owqs_set_angles": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t]),
    "owqs_set_outcomes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint8), ctypes.c_size_t]),
    "owqs_run": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int, _vp]),
    "owqs_read_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int, _vp]),
    "owqs_check": (ctypes.c_int, [_vp, _vp]),
    "owqs_read_probs": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t, _vp]),
    "owqs_set_outcome_seed": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "owqs_get_outcomes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint8), ctypes.c_size_t]),
    "owqs_set_uniforms": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t]),
    "owqs_read_outcomes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint8), ctypes.c_size_t, _vp]),
    "owqs_run_range": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_size_t, ctypes.c_size_t,
                                      _vp]),
    "owqs_read_live": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _i32p, _i32p, _vp]),
    "owqs_set_graph": (ctypes.c_int, [_vp, ctypes.c_int]),
    "owqs_set_tile_bits": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "owqs_set_sum_all": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "owqs_tune": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int, _vp, _i32p,
                                 ctypes.POINTER(ctypes.c_float)]),
    "owqs_plan_info": (ctypes.c_int, [_vp, _i32p, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "owqs_plan_tile_work": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "owqs_run_basis": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _vp, _vp]),
    "owqs_run_states": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _vp, _vp, _vp]),
    "owqs_run_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp, _vp, _vp]),
    "owqs_run_batch": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_size_t, ctypes.POINTER(_vp),
                                      ctypes.POINTER(_vp), _vp]),
    "owqs_tune_batch": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_size_t, ctypes.POINTER(_vp),
                                       ctypes.POINTER(_vp), _vp, _i32p, ctypes.POINTER(ctypes.c_float)]),
    "owqs_adjoint": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t, _i32p,
                                    ctypes.c_int32, _vp, _vp, ctypes.c_int32, _vp]),
    "owqs_pattern_commands": (ctypes.c_int, [_vp, ctypes.POINTER(OwqsCmd), ctypes.c_size_t, _i32p, ctypes.c_size_t,
                                             _i32p, _i32p, ctypes.POINTER(ctypes.c_size_t),
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "owqs_pattern_reorder": (ctypes.c_int, [_vp, ctypes.c_void_p, ctypes.POINTER(_vp), ctypes.c_void_p]),
    "owqs_pattern_certify": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint8), ctypes.c_size_t, _i32p, _i32p]),
    "owqs_pattern_gflow": (ctypes.c_int, [_vp, _i32p, _i32p, _i32p, ctypes.c_size_t]),
    "owqs_set_input_factors": (ctypes.c_int, [_vp, _i32p, ctypes.c_size_t]),
    "owqs_run_factors": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), _i32p, ctypes.c_size_t, ctypes.c_int, _vp]),
    "owqs_read_substates": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _i32p, _i32p, ctypes.c_size_t, _i32p,
                                           ctypes.POINTER(ctypes.c_size_t), _vp, _vp]),
    "owqs_run_profiled": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int, _vp,
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class ProaOpts(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("delta", ctypes.c_double), ("ignore_dependencies", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ProaStats(ctypes.Structure):
    _fields_ = [("max_state_space", ctypes.c_int32), ("max_live", ctypes.c_int32), ("alpha", ctypes.c_double)]


PatternSpec = collections.namedtuple("PatternSpec", "inputs outputs cmds")
_OP_NAMES = {v: k for k, v in OPS.items()}


class OwqsError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        name = _lib.owqs_status_str(status).decode()
        super().__init__(f"{name}: {detail}" if detail else name)
        self.status = status


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Context:
    """A libowqs context bound to one HIP device."""

    def __init__(self, device: int = 0):
        h = _vp()
        st = _lib.owqs_ctx_create(int(device), ctypes.byref(h))
        if st != OK:
            raise OwqsError(st, f"device {device}")
        self._h = h
        self.device = int(device)

    def check(self, status: int):
        if status != OK:
            raise OwqsError(status, _lib.owqs_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib.owqs_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _marshal(pattern):
    cmds = (OwqsCmd * max(len(pattern.cmds), 1))()
    dom = []
    for i, c in enumerate(pattern.cmds):
        x = cmds[i]
        x.op = OPS[c[0]]
        x.q0 = int(c[1])
        if c[0] == "E":
            x.q1 = int(c[2])
        elif c[0] == "M":
            x.angle = float(c[2])
            x.s_off, x.s_len = len(dom), len(c[3])
            dom.extend(int(j) for j in c[3])
            x.t_off, x.t_len = len(dom), len(c[4])
            dom.extend(int(j) for j in c[4])
        elif c[0] in ("X", "Z"):
            x.s_off, x.s_len = len(dom), len(c[2])
            dom.extend(int(j) for j in c[2])
    dom_a = np.array(dom if dom else [0], np.int32)
    ins = np.array(list(pattern.inputs) or [0], np.int32)
    outs = np.array(list(pattern.outputs) or [0], np.int32)
    return cmds, dom_a, len(dom), ins, outs


class Pattern:
    """A pattern loaded into libowqs (owns its device state buffer)."""

    def __init__(self, ctx: Context, pattern=None, text: Optional[str] = None):
        self.ctx = ctx
        h = _vp()
        if text is not None:
            b = text.encode()
            ctx.check(_lib.owqs_pattern_from_text(ctx._h, b, len(b), ctypes.byref(h)))
        else:
            cmds, dom, ndom, ins, outs = _marshal(pattern)
            ctx.check(_lib.owqs_pattern_create(
                ctx._h, cmds, len(pattern.cmds), dom.ctypes.data_as(_i32p), ndom,
                ins.ctypes.data_as(_i32p), len(pattern.inputs), outs.ctypes.data_as(_i32p),
                len(pattern.outputs), ctypes.byref(h)))
        self._adopt(h)

    @classmethod
    def _from_handle(cls, ctx: Context, h) -> "Pattern":
        self = cls.__new__(cls)
        self.ctx = ctx
        self._adopt(h)
        return self

    def _adopt(self, h):
        ctx = self.ctx
        self._h = h
        nm, ml, ni, no = (ctypes.c_int32() for _ in range(4))
        nc = ctypes.c_size_t()
        ctx.check(_lib.owqs_pattern_info(h, ctypes.byref(nm), ctypes.byref(ml), ctypes.byref(ni),
                                         ctypes.byref(no), ctypes.byref(nc)))
        self.n_meas, self.max_live, self.n_in, self.n_out, self.ncmds = nm.value, ml.value, ni.value, no.value, nc.value

    def commands(self) -> PatternSpec:
        """The pattern as loaded (owqs_pattern_commands): inputs, outputs and
        command tuples ("N", q), ("E", u, v), ("M", q, alpha, s, t),
        ("X", q, s), ("Z", q, s) with domains as tuples of qubit ids."""
        nc, nd = ctypes.c_size_t(), ctypes.c_size_t()
        self.ctx.check(_lib.owqs_pattern_commands(self._h, None, 0, None, 0, None, None, ctypes.byref(nc),
                                                  ctypes.byref(nd)))
        cmds = (OwqsCmd * max(nc.value, 1))()
        dom = np.zeros(max(nd.value, 1), np.int32)
        ins = np.zeros(max(self.n_in, 1), np.int32)
        outs = np.zeros(max(self.n_out, 1), np.int32)
        self.ctx.check(_lib.owqs_pattern_commands(self._h, cmds, nc.value, dom.ctypes.data_as(_i32p), dom.size,
                                                  ins.ctypes.data_as(_i32p), outs.ctypes.data_as(_i32p),
                                                  ctypes.byref(nc), ctypes.byref(nd)))

        def rng(off, n):
            return tuple(int(q) for q in dom[off:off + n])

        out = []
        for c in cmds[: nc.value]:
            op = _OP_NAMES[c.op]
            if op == "N":
                out.append(("N", c.q0))
            elif op == "E":
                out.append(("E", c.q0, c.q1))
            elif op == "M":
                out.append(("M", c.q0, c.angle, rng(c.s_off, c.s_len), rng(c.t_off, c.t_len)))
            else:
                out.append((op, c.q0, rng(c.s_off, c.s_len)))
        return PatternSpec([int(q) for q in ins[: self.n_in]], [int(q) for q in outs[: self.n_out]], out)

    def reorder(self, weights: Optional[Sequence[float]] = None, ignore_dependencies: bool = False):
        """PROA (owqs_pattern_reorder): returns (reordered Pattern, stats dict
        with max_state_space, max_live, alpha).  weights = (alpha, beta,
        gamma, delta), or None for the default alpha sweep."""
        opts = ProaOpts()
        if weights is not None:
            opts.alpha, opts.beta, opts.gamma, opts.delta = (float(w) for w in weights)
        opts.ignore_dependencies = 1 if ignore_dependencies else 0
        st = ProaStats()
        h = _vp()
        self.ctx.check(_lib.owqs_pattern_reorder(self._h, ctypes.byref(opts), ctypes.byref(h), ctypes.byref(st)))
        return Pattern._from_handle(self.ctx, h), {"max_state_space": st.max_state_space,
                                                   "max_live": st.max_live, "alpha": st.alpha}

    def certify(self):
        """EOWQS certificate for this order (owqs_pattern_certify): per M,
        whether a gflow witness exists; plus the first M without one (-1)."""
        w = np.zeros(max(self.n_meas, 1), np.uint8)
        nc, fm = ctypes.c_int32(), ctypes.c_int32()
        self.ctx.check(_lib.owqs_pattern_certify(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                                 self.n_meas, ctypes.byref(nc), ctypes.byref(fm)))
        return w[: self.n_meas].astype(bool), fm.value

    def gflow(self):
        """(exists, depth, layer of each M's qubit) of a maximally delayed gflow
        of the open graph (owqs_pattern_gflow)."""
        lay = np.zeros(max(self.n_meas, 1), np.int32)
        ex, dp = ctypes.c_int32(), ctypes.c_int32()
        self.ctx.check(_lib.owqs_pattern_gflow(self._h, ctypes.byref(ex), ctypes.byref(dp),
                                               lay.ctypes.data_as(_i32p), self.n_meas))
        return bool(ex.value), dp.value, lay[: self.n_meas].copy()

    def set_mode(self, mode: int):
        self.ctx.check(_lib.owqs_set_mode(self._h, int(mode)))

    def set_exec(self, exec_: int):
        self.ctx.check(_lib.owqs_set_exec(self._h, int(exec_)))

    def set_graph(self, enable: bool):
        self.ctx.check(_lib.owqs_set_graph(self._h, 1 if enable else 0))

    def set_tile_bits(self, bits: int):
        self.ctx.check(_lib.owqs_set_tile_bits(self._h, int(bits)))

    def set_sum_all(self, on: bool):
        """OWQS: sum every M's probability, also where p = 1/2 exactly."""
        self.ctx.check(_lib.owqs_set_sum_all(self._h, 1 if on else 0))

    def tune(self, psi_in=None, stream=None):
        """Pick the fastest tile size for this pattern; returns (bits, ms per run)."""
        b = ctypes.c_int32()
        t = ctypes.c_float()
        ptr, n = (None, 1) if psi_in is None else (psi_in.data_ptr(), psi_in.numel())
        self.ctx.check(_lib.owqs_tune(self._h, ptr, n, 1, _stream_handle(stream), ctypes.byref(b), ctypes.byref(t)))
        return b.value, t.value

    def plan_info(self):
        """(plan width, steps, passes over global memory) for the current settings."""
        w = ctypes.c_int32()
        n = ctypes.c_size_t()
        x = ctypes.c_size_t()
        self.ctx.check(_lib.owqs_plan_info(self._h, ctypes.byref(w), ctypes.byref(n), ctypes.byref(x)))
        return w.value, n.value, x.value

    def plan_tile_work(self):
        """(windows applied one by one, composed 2x2 maps, windows inside the
        maps) of the fused plan's tile passes, forced outcomes, no window sums."""
        w = ctypes.c_size_t()
        m = ctypes.c_size_t()
        c = ctypes.c_size_t()
        self.ctx.check(_lib.owqs_plan_tile_work(self._h, ctypes.byref(w), ctypes.byref(m), ctypes.byref(c)))
        return w.value, m.value, c.value

    def run_basis(self, first: int = 0, count: Optional[int] = None, out=None, probs=None, stream=None):
        """Outputs for basis inputs |first> .. |first+count-1> as a
        (count, 2^n_out) complex64 CUDA tensor (row k = output for |first+k>)."""
        import torch
        if count is None:
            count = (1 << self.n_in) - first
        if out is None:
            out = torch.empty((count, 1 << self.n_out), dtype=torch.complex64, device=f"cuda:{self.ctx.device}")
        self._check_out(out, count << self.n_out)
        pp = None if probs is None else probs.data_ptr()
        self.ctx.check(_lib.owqs_run_basis(self._h, int(first), int(count), out.data_ptr(), pp,
                                           _stream_handle(stream)))
        return out

    def run_states(self, states, out=None, probs=None, stream=None):
        """Outputs for a (count, 2^n_in) complex64 CUDA tensor of input states."""
        import torch
        if states.dtype != torch.complex64 or not states.is_cuda or not states.is_contiguous():
            raise TypeError("states must be a contiguous complex64 CUDA tensor")
        count = states.numel() >> self.n_in
        if out is None:
            out = torch.empty((count, 1 << self.n_out), dtype=torch.complex64, device=f"cuda:{self.ctx.device}")
        self._check_out(out, count << self.n_out)
        pp = None if probs is None else probs.data_ptr()
        self.ctx.check(_lib.owqs_run_states(self._h, states.data_ptr(), int(count), out.data_ptr(), pp,
                                            _stream_handle(stream)))
        return out

    def run_noalloc(self, psi_in, out, probs=None, err=None, stream=None):
        """owqs_run_noalloc: the whole run with the library's fixed working
        array (no device allocation).  psi_in: complex64 CUDA tensor of
        2^n_in amplitudes or None (n_in = 0); out: complex64 CUDA tensor of
        2^n_out; probs: float64 CUDA tensor of n_meas or None; err: int32
        CUDA tensor of 2 or None.  Returns out."""
        import torch
        self._check_out(out, 1 << self.n_out)
        if psi_in is None:
            ip, n_in = None, 1
        else:
            if psi_in.dtype != torch.complex64 or not psi_in.is_cuda or not psi_in.is_contiguous():
                raise TypeError("input must be a contiguous complex64 CUDA tensor")
            ip, n_in = psi_in.data_ptr(), psi_in.numel()
        if probs is not None and (probs.dtype != torch.float64 or not probs.is_cuda or probs.numel() != self.n_meas):
            raise TypeError("probs must be a float64 CUDA tensor of n_meas entries")
        if err is not None and (err.dtype != torch.int32 or not err.is_cuda or err.numel() != 2):
            raise TypeError("err must be an int32 CUDA tensor of 2 entries")
        self.ctx.check(_lib.owqs_run_noalloc(self._h, ip, n_in, out.data_ptr(), out.numel(),
                                             None if probs is None else probs.data_ptr(),
                                             None if err is None else err.data_ptr(), _stream_handle(stream)))
        return out

    @staticmethod
    def _check_out(out, n):
        import torch
        if out.dtype != torch.complex64 or not out.is_cuda or not out.is_contiguous() or out.numel() != n:
            raise TypeError("output must be a contiguous complex64 CUDA tensor of the right size")

    def adjoint(self, alphas, obs: Optional[Sequence[int]] = None, psi_in=None, ckpt_stride: int = 0,
                stream=None):
        """Loss sum_i <Z_obs[i]> (EOWQS) and its gradient for a (B, n_meas)
        array of M angles: returns (loss (B,), grad (B, n_meas)) as float64
        CUDA tensors."""
        import torch
        a = np.ascontiguousarray(np.asarray(alphas, np.float64).reshape(-1, self.n_meas))
        batch = a.shape[0]
        obs_l = list(range(self.n_out)) if obs is None else [int(o) for o in obs]
        ob = np.array(obs_l or [0], np.int32)
        dev = f"cuda:{self.ctx.device}"
        loss = torch.empty(batch, dtype=torch.float64, device=dev)
        grad = torch.empty((batch, self.n_meas), dtype=torch.float64, device=dev)
        ptr = None
        if psi_in is not None:
            if psi_in.dtype != torch.complex64 or not psi_in.is_cuda or not psi_in.is_contiguous():
                raise TypeError("input must be a contiguous complex64 CUDA tensor")
            ptr = psi_in.data_ptr()
        self.ctx.check(_lib.owqs_adjoint(
            self._h, ptr, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), batch, ob.ctypes.data_as(_i32p),
            len(obs_l), loss.data_ptr(), grad.data_ptr(), int(ckpt_stride), _stream_handle(stream)))
        return loss, grad

    def set_angles(self, alphas: Sequence[float]):
        a = np.ascontiguousarray(alphas, np.float64)
        self.ctx.check(_lib.owqs_set_angles(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.size))

    def set_outcomes(self, bits: Sequence[int]):
        b = np.ascontiguousarray(bits, np.uint8)
        self.ctx.check(_lib.owqs_set_outcomes(self._h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), b.size))

    def set_outcome_seed(self, seed: int):
        """Outcomes from the SplitMix64 bit stream of `seed` (owqs_set_outcome_seed)."""
        self.ctx.check(_lib.owqs_set_outcome_seed(self._h, int(seed) & (2**64 - 1)))

    def outcomes(self) -> np.ndarray:
        b = np.zeros(max(self.n_meas, 1), np.uint8)
        self.ctx.check(_lib.owqs_get_outcomes(self._h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), self.n_meas))
        return b[: self.n_meas]

    def set_uniforms(self, u):
        """Draw outcomes on the device from these uniforms (owqs_set_uniforms);
        None returns to forced outcomes."""
        if u is None:
            self.ctx.check(_lib.owqs_set_uniforms(self._h, None, 0))
            return
        a = np.ascontiguousarray(u, np.float64)
        self.ctx.check(_lib.owqs_set_uniforms(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.size))

    def read_outcomes(self, stream=None) -> np.ndarray:
        """Outcomes of the last run (drawn or forced)."""
        b = np.zeros(max(self.n_meas, 1), np.uint8)
        h = None if self.ctx.device < 0 else _stream_handle(stream)  # a host-only context has no stream
        self.ctx.check(_lib.owqs_read_outcomes(self._h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                               self.n_meas, h))
        return b[: self.n_meas]

    def run_range(self, begin: int, end: int, psi_in=None, stream=None):
        """Run commands [begin, end) with the plain plan (owqs_run_range); begin = 0
        starts from psi_in (complex64 CUDA tensor, None when n_in = 0)."""
        ptr, n = None, 1
        if psi_in is not None:
            import torch
            if psi_in.dtype != torch.complex64 or not psi_in.is_cuda or not psi_in.is_contiguous():
                raise TypeError("input must be a contiguous complex64 CUDA tensor")
            ptr, n = psi_in.data_ptr(), psi_in.numel()
        elif begin == 0 and self.n_in:
            raise ValueError("this pattern needs an input state")
        self.ctx.check(_lib.owqs_run_range(self._h, ptr, n, 1, int(begin), int(end), _stream_handle(stream)))

    def read_live(self, stream=None):
        """After run_range: (live vector as complex64 numpy array, caller qubit id of each bit)."""
        q = np.zeros(MAX_WIDTH, np.int32)
        nl = np.zeros(1, np.int32)
        i32 = ctypes.POINTER(ctypes.c_int32)
        self.ctx.check(_lib.owqs_read_live(self._h, None, 0, q.ctypes.data_as(i32), nl.ctypes.data_as(i32),
                                           _stream_handle(stream)))
        n = int(nl[0])
        out = np.zeros(1 << n, np.complex64)
        self.ctx.check(_lib.owqs_read_live(self._h, out.ctypes.data, out.size, q.ctypes.data_as(i32),
                                           nl.ctypes.data_as(i32), _stream_handle(stream)))
        return out, [int(x) for x in q[:n]]

    def run(self, psi_in=None, stream=None):
        """psi_in: complex64 CUDA tensor of 2^n_in amplitudes (None when n_in = 0)."""
        if psi_in is None:
            if self.n_in:
                raise ValueError("this pattern needs an input state")
            self.ctx.check(_lib.owqs_run(self._h, None, 1, 1, _stream_handle(stream)))
            return
        import torch
        if psi_in.dtype != torch.complex64 or not psi_in.is_cuda or not psi_in.is_contiguous():
            raise TypeError("input must be a contiguous complex64 CUDA tensor")
        self.ctx.check(_lib.owqs_run(self._h, psi_in.data_ptr(), psi_in.numel(), 1, _stream_handle(stream)))

    def set_input_factors(self, factor_nq: Sequence[int]):
        """Split the inputs into initial sub-states of these sizes (input order)."""
        a = np.array(list(factor_nq) or [0], np.int32)
        self.ctx.check(_lib.owqs_set_input_factors(self._h, a.ctypes.data_as(_i32p), len(factor_nq)))

    def run_factors(self, factors, stream=None):
        """Sub-state executor: run with the input as a tensor product of
        complex64 CUDA tensors, factor k over the next log2(len) inputs
        (owqs_run_factors)."""
        import torch
        for f in factors:
            if f.dtype != torch.complex64 or not f.is_cuda or not f.is_contiguous():
                raise TypeError("factors must be contiguous complex64 CUDA tensors")
        nq = np.array([max(int(f.numel()).bit_length() - 1, 0) for f in factors] or [0], np.int32)
        ptrs = (_vp * max(len(factors), 1))(*[f.data_ptr() for f in factors])
        self.ctx.check(_lib.owqs_run_factors(self._h, ptrs, nq.ctypes.data_as(_i32p), len(factors), 1,
                                             _stream_handle(stream)))

    def read_substates(self, stream=None):
        """After a sub-state run: ([(qubit ids, complex64 numpy vector), ...],
        complex scalar) with the output state = scalar x the tensor product
        (owqs_read_substates)."""
        nf = ctypes.c_int32()
        na = ctypes.c_size_t()
        h = _stream_handle(stream)
        self.ctx.check(_lib.owqs_read_substates(self._h, None, 0, None, None, 0, ctypes.byref(nf), ctypes.byref(na),
                                                None, h))
        fq = np.zeros(max(nf.value, 1), np.int32)
        qs = np.zeros(max(self.n_out, 1), np.int32)
        amps = np.zeros(max(na.value, 1), np.complex64)
        sc = np.zeros(1, np.complex64)
        self.ctx.check(_lib.owqs_read_substates(self._h, amps.ctypes.data, amps.size, fq.ctypes.data_as(_i32p),
                                                qs.ctypes.data_as(_i32p), fq.size, ctypes.byref(nf),
                                                ctypes.byref(na), sc.ctypes.data, h))
        out, a, q = [], 0, 0
        for f in range(nf.value):
            k = int(fq[f])
            out.append(([int(x) for x in qs[q:q + k]], amps[a:a + (1 << k)].copy()))
            a += 1 << k
            q += k
        return out, complex(sc[0])

    def run_profiled(self, psi_in=None, stream=None) -> dict:
        """Run once with HIP events between launches; returns, per kernel kind,
        {"launches", "ms", "bytes"} (algorithmic bytes, element level)."""
        counts = np.zeros(NUM_KINDS, np.int64)
        ms = np.zeros(NUM_KINDS, np.float64)
        by = np.zeros(NUM_KINDS, np.float64)
        ptr, n = None, 1
        if psi_in is not None:
            ptr, n = psi_in.data_ptr(), psi_in.numel()
        elif self.n_in:
            raise ValueError("this pattern needs an input state")
        self.ctx.check(_lib.owqs_run_profiled(
            self._h, ptr, n, 1, _stream_handle(stream), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), by.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return {KINDS[k]: {"launches": int(counts[k]), "ms": float(ms[k]), "bytes": float(by[k])}
                for k in KINDS if counts[k]}

    def read_state(self, out=None, stream=None, check: bool = True):
        """Output state as a complex64 CUDA tensor (outputs[k] at bit k)."""
        import torch
        n = 1 << self.n_out
        if out is None:
            out = torch.empty(n, dtype=torch.complex64, device=f"cuda:{self.ctx.device}")
        if out.numel() != n or out.dtype != torch.complex64 or not out.is_contiguous():
            raise TypeError("output must be a contiguous complex64 tensor of 2^n_out entries")
        self.ctx.check(_lib.owqs_read_state(self._h, out.data_ptr(), n, 1, _stream_handle(stream)))
        if check:
            self.check(stream)
        return out

    def check(self, stream=None):
        self.ctx.check(_lib.owqs_check(self._h, _stream_handle(stream)))

    def read_probs(self, stream=None) -> np.ndarray:
        p = np.zeros(max(self.n_meas, 1), np.float64)
        self.ctx.check(_lib.owqs_read_probs(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            self.n_meas, _stream_handle(stream)))
        return p[: self.n_meas]

    def close(self):
        if getattr(self, "_h", None):
            _lib.owqs_pattern_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_batch(ctx: Context, patterns: Sequence["Pattern"], inputs, outputs, stream=None):
    """owqs_tune_batch: the fastest tile size for a batch; returns (bits, ms per call)."""
    n = len(patterns)
    ph = (_vp * max(n, 1))(*[p._h for p in patterns])
    ih = (_vp * max(n, 1))(*[None if x is None else x.data_ptr() for x in inputs])
    oh = (_vp * max(n, 1))(*[o.data_ptr() for o in outputs])
    bits = ctypes.c_int32(0)
    ms = ctypes.c_float(0.0)
    ctx.check(_lib.owqs_tune_batch(ctx._h, ph, n, ih, oh, _stream_handle(stream), ctypes.byref(bits),
                                   ctypes.byref(ms)))
    return int(bits.value), float(ms.value)


def run_batch(ctx: Context, patterns: Sequence["Pattern"], inputs, outputs, stream=None):
    """Run loaded patterns as one batch (owqs_run_batch).  inputs[i] is a
    complex64 CUDA tensor or None; outputs[i] a complex64 CUDA tensor."""
    n = len(patterns)
    ph = (_vp * max(n, 1))(*[p._h for p in patterns])
    ih = (_vp * max(n, 1))(*[None if x is None else x.data_ptr() for x in inputs])
    oh = (_vp * max(n, 1))(*[o.data_ptr() for o in outputs])
    ctx.check(_lib.owqs_run_batch(ctx._h, ph, n, ih, oh, _stream_handle(stream)))


def _make_loss_function():
    import torch

    class PatternLoss(torch.autograd.Function):
        """L_b = sum_i <Z_obs[i]> of the pattern's output for each row b of
        the (B, n_meas) angle tensor; the gradient comes from owqs_adjoint
        (computed together with the loss in the forward call)."""

        @staticmethod
        def forward(ctx, alphas, pattern, obs, psi_in, ckpt_stride):
            a = alphas.detach().to("cpu", torch.float64).numpy()
            loss, grad = pattern.adjoint(a, obs, psi_in, ckpt_stride)
            ctx.save_for_backward(grad)
            ctx.in_dtype = alphas.dtype
            ctx.in_device = alphas.device
            return loss.to(device=alphas.device, dtype=alphas.dtype)

        @staticmethod
        def backward(ctx, gout):
            (grad,) = ctx.saved_tensors
            g = gout.to(grad.device, grad.dtype)[:, None] * grad
            return g.to(device=ctx.in_device, dtype=ctx.in_dtype), None, None, None, None

    return PatternLoss


PatternLoss = _make_loss_function()


def pattern_loss(pattern: "Pattern", alphas, obs=None, psi_in=None, ckpt_stride: int = 0):
    """Differentiable loss: ``pattern_loss(p, alphas).sum().backward()`` fills
    ``alphas.grad`` with the adjoint gradient."""
    return PatternLoss.apply(alphas, pattern, obs, psi_in, ckpt_stride)


def run_pattern(ctx: Context, pattern, outcomes, input_state=None, mode: int = MODE_OWQS,
                exec_: int = EXEC_AUTO, angles=None):
    """Load, run and read one pattern; returns (output complex64 CUDA tensor, probs)."""
    import torch
    p = Pattern(ctx, pattern)
    try:
        p.set_mode(mode)
        p.set_exec(exec_)
        if angles is not None:
            p.set_angles(angles)
        p.set_outcomes(outcomes)
        x = None
        if input_state is not None:
            x = torch.as_tensor(np.asarray(input_state, np.complex64)).to(f"cuda:{ctx.device}")
        p.run(x)
        out = p.read_state()
        probs = p.read_probs()
        torch.cuda.synchronize()
        return out, probs
    finally:
        p.close()
