"""ctypes binding of libsv.so (include/sv.h and include/sv_host.h).

Argument marshalling only: every step of the simulation runs in the HIP
library.  Device memory for states comes from PyTorch (a complex tensor on
the GPU that the library wraps with ``sv_attach``), and work is enqueued on
PyTorch's current stream.  Importing this module fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsv.so")

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_ERANGE, SV_ESTATE = 0, -1, -2, -3, -4, -5
C64, C128 = 0, 1
MODES = {"plain": 0, "spec": 1, "fused": 2, "tiled": 3, "regtile": 4, "auto": 5}
SWEEP_KINDS = {1: "init", 2: "plain_1q", 3: "plain_cz", 4: "spec_dense", 5: "spec_real",
               6: "spec_diag", 7: "spec_cz", 8: "regtile", 9: "ldstile", 10: "ldstile_mfma"}


class SVError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("sv status %d: %s" % (status, msg))
        self.status = status


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("cycle", ctypes.c_int32), ("param", ctypes.c_int32), ("mat", ctypes.c_int32)]


class CCircuit(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nparams", ctypes.c_int32), ("ngates", ctypes.c_int64),
                ("gates", ctypes.c_void_p), ("theta", ctypes.c_void_p), ("nmats", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("mats", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("k_max", ctypes.c_int32),
                ("tile_qubits", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("sweep_budget", ctypes.c_int32), ("checkpoint_c", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double), ("entropy", ctypes.c_double),
                ("unif_ce", ctypes.c_double), ("moments", ctypes.c_double * 10),
                ("zero_count", ctypes.c_int64)]

    def as_dict(self) -> dict:
        d = {"norm": self.norm, "entropy": self.entropy, "unif_ce": self.unif_ce,
             "zero_count": int(self.zero_count)}
        m = np.array(list(self.moments))
        for k in range(10):
            d["M%d" % (k + 1)] = float(m[k])
        d["moments"] = m
        return d


class Pair(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("norm_a", "norm_b", "overlap_re", "overlap_im", "fidelity",
                                               "xent", "unif_ce", "delta_h", "corr", "zero_mass_b")] + \
               [("zero_a", ctypes.c_int64)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["zero_a"] = int(self.zero_a)
        return d


EXPORTS = {
    # name: (restype, argtypes)
    "sv_alloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "sv_attach": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p]),
    "sv_free": (ctypes.c_int, [ctypes.c_void_p]),
    "sv_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "sv_data": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sv_apply_circuit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sv_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "sv_probs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                ctypes.c_void_p]),
    "sv_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sv_cycle_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "sv_host_cycle_emulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "sv_sample": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p,
                                 ctypes.c_int]),
    "sv_moments_sample": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                                         ctypes.c_void_p, ctypes.c_int]),
    "sv_moments_sample_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                 ctypes.c_uint64, ctypes.c_void_p]),
    "sv_pair_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    "sv_sample_from": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "sv_cross_entropy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sv_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p]),
    "sv_apply_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "sv_last_error": (ctypes.c_char_p, []),
    "sv_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p]),
    "sv_apply_circuit_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p]),
    "sv_host_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sv_host_emulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p]),
    "sv_host_plan_describe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_char_p, ctypes.c_int64]),
}

_lib = None


def lib():
    """The loaded library; raises if it is missing (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsv.so is not built (run __graft_entry__.build() or "
                              "python paper_1608_00263_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != SV_OK:
        raise SVError(status, lib().sv_last_error().decode(errors="replace"))


def _ptr(a) -> Optional[int]:
    return a.ctypes.data if a is not None and a.size else None


class CircuitArgs:
    """Holds an sv_circuit and the arrays it points to."""

    def __init__(self, circ):
        g = circ.gates
        self.gates = np.ascontiguousarray(
            np.stack([g[f] for f in ("kind", "q0", "q1", "cycle", "param", "mat")], axis=1)
            .astype(np.int32))
        self.theta = np.ascontiguousarray(circ.theta, dtype=np.float64)
        self.mats = np.ascontiguousarray(np.asarray(circ.mats, dtype=np.complex128)).view(np.float64)
        self.c = CCircuit(circ.n, self.theta.size, self.gates.shape[0], _ptr(self.gates),
                          _ptr(self.theta), self.mats.size // 8, 0, _ptr(self.mats))

    @property
    def ref(self):
        return ctypes.byref(self.c)


FLAG_FROM_ZERO = 1
FLAG_NO_MFMA = 2
FLAG_STATE_READY = 4
FLAG_BATCH_LAUNCHES = 8
FLAG_BATCH_PERSISTENT = 16
FLAG_CHECKPOINTS = 32


def make_opts(mode="auto", k_max=0, tile=0, from_zero=False, no_mfma=False, flags=0, budget=0,
              checkpoint_c=0) -> Opts:
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    return Opts(m, k_max, tile, (FLAG_FROM_ZERO if from_zero else 0) | (FLAG_NO_MFMA if no_mfma else 0) | flags,
                budget, checkpoint_c)


def _stream_handle(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class State:
    """A 2^n state on the GPU: a torch tensor wrapped by an sv_state handle."""

    def __init__(self, n: int, dtype: str = "c64", device: str = "cuda:0", tensor=None):
        import torch
        self.torch = torch
        self.n = n
        self.dt = C64 if dtype == "c64" else C128
        tdt = torch.complex64 if self.dt == C64 else torch.complex128
        if tensor is None:
            tensor = torch.zeros(1 << n, dtype=tdt, device=device)
        assert tensor.dtype == tdt and tensor.numel() == (1 << n) and tensor.is_contiguous()
        self.tensor = tensor
        h = ctypes.c_void_p()
        check(lib().sv_attach(n, self.dt, ctypes.c_void_p(tensor.data_ptr()),
                              _stream_handle(torch), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().sv_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        check(lib().sv_reset(self.h))

    def apply(self, circ, mode="auto", k_max=0, tile=0, args: Optional[CircuitArgs] = None,
              from_zero=False, no_mfma=False, budget=0):
        """Apply circ in place (from |0..0> regardless of contents if from_zero)."""
        a = args or CircuitArgs(circ)
        o = make_opts(mode, k_max, tile, from_zero, no_mfma, budget=budget)
        check(lib().sv_apply_circuit(self.h, a.ref, ctypes.byref(o)))

    def forward_checkpoints(self, circ, checkpoint_c: int, tile=0, budget=0,
                            args: Optional[CircuitArgs] = None):
        """U|0..0> as the forward pass of backward(): the state copies of
        every checkpoint_c cycles are kept, so that backward(...,
        checkpoint_c, state_ready=True) with the same circuit and options
        skips the forward."""
        a = args or CircuitArgs(circ)
        o = make_opts("regtile", 0, tile, flags=FLAG_CHECKPOINTS, budget=budget, checkpoint_c=checkpoint_c)
        check(lib().sv_apply_circuit(self.h, a.ref, ctypes.byref(o)))

    def apply_timed(self, circ, mode="auto", k_max=0, tile=0, args: Optional[CircuitArgs] = None,
                    from_zero=False, budget=0):
        """Apply with per-sweep HIP event timing; returns (ms, kinds, bytes) arrays."""
        a = args or CircuitArgs(circ)
        o = make_opts(mode, k_max, tile, from_zero, budget=budget)
        cap = 4096
        ms = np.zeros(cap, dtype=np.float32)
        kinds = np.zeros(cap, dtype=np.int32)
        by = np.zeros(cap, dtype=np.float64)
        n = ctypes.c_int64()
        check(lib().sv_apply_circuit_timed(self.h, a.ref, ctypes.byref(o), cap, _ptr(ms), _ptr(kinds),
                                           _ptr(by), ctypes.byref(n)))
        m = min(n.value, cap)
        return ms[:m], kinds[:m], by[:m]

    def autotune(self, circ, from_zero=True):
        """Run the autotuner for circ; returns (mode name, k_max, tile, complete,
        sweep budget)."""
        a = CircuitArgs(circ)
        o = Opts()
        done = ctypes.c_int()
        check(lib().sv_autotune(self.h, a.ref, 1 if from_zero else 0, ctypes.byref(o), ctypes.byref(done)))
        name = {v: k for k, v in MODES.items()}[o.mode]
        return name, o.k_max, o.tile_qubits, bool(done.value), o.sweep_budget

    def plan_info(self, circ, mode="auto", k_max=0, tile=0, no_mfma=False, budget=0, from_zero=False):
        """(sweeps, algorithmic bytes) of the plan apply() runs with the same
        arguments."""
        a = CircuitArgs(circ)
        o = make_opts(mode, k_max, tile, from_zero=from_zero, no_mfma=no_mfma, budget=budget)
        sw = ctypes.c_int64()
        by = ctypes.c_double()
        check(lib().sv_plan_info(self.h, a.ref, ctypes.byref(o), ctypes.byref(sw), ctypes.byref(by)))
        return sw.value, by.value

    def amplitudes(self) -> np.ndarray:
        self.torch.cuda.synchronize()
        return self.tensor.cpu().numpy()

    def probs(self, begin: int = 0, count: Optional[int] = None, f64: bool = True):
        torch = self.torch
        count = (1 << self.n) - begin if count is None else count
        out = torch.empty(max(count, 1), dtype=torch.float64 if f64 else torch.float32,
                          device=self.tensor.device)
        check(lib().sv_probs(self.h, begin, count, 1 if f64 else 0, ctypes.c_void_p(out.data_ptr())))
        return out[:count]

    def moments(self) -> dict:
        s = Stats()
        check(lib().sv_moments(self.h, ctypes.byref(s)))
        return s.as_dict()

    def cycle_moments(self, circ, mode="auto", tile=0, budget=0, args: Optional[CircuitArgs] = None):
        """Statistics after every cycle 0..D of circ run from |0..0> (a list
        of dicts, one per cycle); the state ends as the circuit's output."""
        a = args or CircuitArgs(circ)
        o = make_opts(mode, 0, tile, from_zero=True, budget=budget)
        D = int(circ.gates["cycle"].max()) if circ.ngates else 0
        out = (Stats * (D + 1))()
        nc = ctypes.c_int64()
        check(lib().sv_cycle_moments(self.h, a.ref, ctypes.byref(o), D + 1, out, ctypes.byref(nc)))
        return [s.as_dict() for s in out[:nc.value]]

    def sample(self, k: int, seed: int) -> np.ndarray:
        out = np.zeros(max(k, 1), dtype=np.uint64)
        check(lib().sv_sample(self.h, k, ctypes.c_uint64(seed), _ptr(out), 0))
        return out[:k]

    def moments_and_sample(self, k: int, seed: int):
        """(moments(), sample(k, seed)) from one read of the state."""
        s = Stats()
        out = np.zeros(max(k, 1), dtype=np.uint64)
        check(lib().sv_moments_sample(self.h, ctypes.byref(s), k, ctypes.c_uint64(seed), _ptr(out), 0))
        return s.as_dict(), out[:k]

    def cross_entropy(self, samples: np.ndarray, norm=None):
        """(ce, delta_h, zero_samples) of the samples; norm, when given, is
        the state's sum of probabilities (moments()["norm"] of the same
        state), which saves the pass that computes it."""
        x = np.ascontiguousarray(samples, dtype=np.uint64)
        ce = ctypes.c_double()
        dh = ctypes.c_double()
        z = ctypes.c_int64()
        check(lib().sv_cross_entropy(self.h, _ptr(x), x.size, 0.0 if norm is None else float(norm),
                                     ctypes.byref(ce), ctypes.byref(dh), ctypes.byref(z)))
        return ce.value, dh.value, z.value

    def backward(self, circ, samples: np.ndarray, checkpoint_c: int = 0, mode="auto", k_max=0,
                 tile=0, state_ready=False, budget=0, args: Optional[CircuitArgs] = None):
        """Loss and adjoint gradient; state_ready=True reuses the output state
        the handle holds (left by apply() of the same circuit, or with
        checkpoint_c > 0 by forward_checkpoints() with the same arguments)
        instead of recomputing it.  args: the circuit marshalled once
        (CircuitArgs(circ)) for repeated calls."""
        a = args or CircuitArgs(circ)
        o = make_opts(mode, k_max, tile, flags=FLAG_STATE_READY if state_ready else 0, budget=budget)
        x = np.ascontiguousarray(samples, dtype=np.uint64)
        grad = np.zeros(max(circ.nparams, 1))
        loss = ctypes.c_double()
        check(lib().sv_backward(self.h, a.ref, ctypes.byref(o), _ptr(x), x.size, checkpoint_c,
                                ctypes.byref(loss), _ptr(grad)))
        return loss.value, grad[:circ.nparams]


def pair_stats(a: "State", b: "State", nbins: int = 0, zmin: float = -8.0, zmax: float = 4.0):
    """Pair statistics of the ideal output a and another output b: a dict
    (sv_pair fields) and, for nbins > 0, the histogram of z = ln(N p_a) as a
    (3, nbins + 2) uint64 array (counts, integer masses of p_a and p_b)."""
    out = Pair()
    hist = np.zeros(3 * (nbins + 2) if nbins > 0 else 1, dtype=np.uint64)
    check(lib().sv_pair_stats(a.h, b.h, nbins, zmin, zmax, ctypes.byref(out),
                              _ptr(hist) if nbins > 0 else None))
    return out.as_dict(), (hist.reshape(3, nbins + 2) if nbins > 0 else None)


def sample_from(probs, words, torch=None):
    """Sampler on an explicit distribution (device tensors in, device out)."""
    import torch as _t
    torch = torch or _t
    out = torch.empty(max(words.numel(), 1), dtype=torch.int64, device=probs.device)
    check(lib().sv_sample_from(ctypes.c_void_p(probs.data_ptr()), probs.numel(),
                               ctypes.c_void_p(words.data_ptr()), words.numel(),
                               ctypes.c_void_p(out.data_ptr()), _stream_handle(torch)))
    return out[:words.numel()]


class BatchArgs:
    """Marshalled circuits of an ensemble (reusable across calls)."""

    def __init__(self, circuits):
        self.args = [CircuitArgs(c) for c in circuits]
        self.arr = (CCircuit * len(self.args))(*[a.c for a in self.args])


def apply_batch(states, circuits, mode="auto", k_max=0, tile=0, launches=False,
                persistent=False, args: Optional[BatchArgs] = None):
    """Simulate each circuit from |0..0> into its state; returns per-instance
    stats.  Default schedule: one launch per sweep round over all instances;
    persistent=True: one persistent launch with a work queue; launches=True:
    the ordinary per-instance launches."""
    ba = args or BatchArgs(circuits)      # keeps the gate arrays alive during the call
    hs = (ctypes.c_void_p * len(states))(*[s.h.value for s in states])
    out = (Stats * len(states))()
    o = make_opts(mode, k_max, tile, flags=(FLAG_BATCH_LAUNCHES if launches else 0)
                  | (FLAG_BATCH_PERSISTENT if persistent else 0))
    check(lib().sv_apply_batch(hs, ba.arr, len(states), ctypes.byref(o), out))
    return [s.as_dict() for s in out]


# ---- host-only diagnostics (no GPU) -----------------------------------------
def host_plan(circ, dtype="c64", mode="auto", k_max=0, tile=0, from_zero=True, budget=0, no_mfma=False):
    a = CircuitArgs(circ)
    o = make_opts(mode, k_max, tile, no_mfma=no_mfma, budget=budget)
    sw = ctypes.c_int64()
    by = ctypes.c_double()
    mf = ctypes.c_int64()
    check(lib().sv_host_plan(a.ref, C64 if dtype == "c64" else C128, ctypes.byref(o),
                             1 if from_zero else 0, ctypes.byref(sw), ctypes.byref(by),
                             ctypes.byref(mf)))
    return {"sweeps": sw.value, "bytes": by.value, "mfma_sweeps": mf.value}


def host_emulate(circ, psi: np.ndarray, dtype="c64", mode="auto", k_max=0, tile=0,
                 from_zero=True, budget=0) -> np.ndarray:
    a = CircuitArgs(circ)
    o = make_opts(mode, k_max, tile, budget=budget)
    psi = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    check(lib().sv_host_emulate(a.ref, C64 if dtype == "c64" else C128, ctypes.byref(o),
                                1 if from_zero else 0, _ptr(psi)))
    return psi


def host_cycle_emulate(circ, dtype="c64", mode="auto", tile=0, budget=0):
    """(probabilities at each statistics point of the per-cycle plan, rows x
    2^n; the row reporting each cycle)."""
    a = CircuitArgs(circ)
    o = make_opts(mode, 0, tile, from_zero=True, budget=budget)
    nr = ctypes.c_int64()
    nc = ctypes.c_int64()
    dt = C64 if dtype == "c64" else C128
    rc = lib().sv_host_cycle_emulate(a.ref, dt, ctypes.byref(o), 0, None, None, 0, ctypes.byref(nr),
                                     ctypes.byref(nc))
    if rc not in (SV_OK, SV_ERANGE):
        check(rc)
    probs = np.zeros((nr.value, 1 << circ.n))
    rows = np.zeros(nc.value, dtype=np.int32)
    check(lib().sv_host_cycle_emulate(a.ref, dt, ctypes.byref(o), nr.value, _ptr(probs), _ptr(rows),
                                      nc.value, None, None))
    return probs, rows


def host_plan_describe(circ, dtype="c64", mode="auto", k_max=0, tile=0, from_zero=True,
                       budget=0, no_mfma=False) -> str:
    a = CircuitArgs(circ)
    o = make_opts(mode, k_max, tile, no_mfma=no_mfma, budget=budget)
    buf = ctypes.create_string_buffer(1 << 20)
    check(lib().sv_host_plan_describe(a.ref, C64 if dtype == "c64" else C128, ctypes.byref(o),
                                      1 if from_zero else 0, buf, len(buf)))
    return buf.value.decode()
