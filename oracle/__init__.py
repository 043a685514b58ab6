"""Python front end of the FP64 reference implementation (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the library.  It takes
plain numpy inputs (gate records as an (G, 6) int32 array, amplitudes as
complex128) and shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
EULER_GAMMA = 0.57721566490153286061


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, u64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        L.orc_gate_matrix.argtypes = [i32, f64, P, P]
        L.orc_init_zero.argtypes = [i32, P]
        L.orc_apply_range.argtypes = [i32, P, i64, i64, P, i32, P, i32, P]
        L.orc_apply_circuit.argtypes = [i32, P, i64, P, i32, P, i32, P]
        L.orc_probs.argtypes = [i32, P, P]
        L.orc_probs_c64.argtypes = [i32, P, P]
        L.orc_stats.argtypes = [i32, P, P]
        L.orc_splitmix64.argtypes = [u64, u64]
        L.orc_splitmix64.restype = u64
        L.orc_sample_from_words.argtypes = [u64, P, P, i64, P]
        L.orc_sample.argtypes = [u64, P, u64, i64, P]
        L.orc_cross_entropy.argtypes = [i32, P, P, i64, P, P]
        L.orc_cross_entropy.restype = i64
        L.orc_adjoint.argtypes = [i32, P, i64, P, i32, P, i32, P, i64, P, P]
        L.orc_pair_stats.argtypes = [i32, P, P, i32, f64, f64, P, P]
        L.orc_num_threads.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def _circuit_arrays(circ):
    g = np.ascontiguousarray(
        np.stack([circ.gates[f] for f in ("kind", "q0", "q1", "cycle", "param", "mat")],
                 axis=1).astype(np.int32))
    theta = np.ascontiguousarray(circ.theta, dtype=np.float64)
    mats = np.ascontiguousarray(np.asarray(circ.mats, dtype=np.complex128)).view(np.float64)
    return g, theta, mats


def gate_matrix(kind: int, theta: float = 0.0, mat=None) -> np.ndarray:
    out = np.zeros(8)
    m = None if mat is None else np.ascontiguousarray(mat, dtype=np.complex128).view(np.float64)
    rc = lib().orc_gate_matrix(kind, float(theta), _ptr(m), _ptr(out))
    if rc:
        raise ValueError("unknown gate kind %d" % kind)
    return out.view(np.complex128).reshape(2, 2)


def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_init_zero(n, _ptr(psi))
    return psi


def apply_circuit(circ, psi=None, first: int = 0, last=None) -> np.ndarray:
    """Apply gates [first, last) to psi (|0..0> when None); returns psi."""
    n = circ.n
    if psi is None:
        psi = zero_state(n)
    assert psi.dtype == np.complex128 and psi.shape == (1 << n,) and psi.flags.c_contiguous
    g, theta, mats = _circuit_arrays(circ)
    last = circ.ngates if last is None else last
    rc = lib().orc_apply_range(n, _ptr(g), first, last, _ptr(theta), theta.size,
                               _ptr(mats), mats.size // 8, _ptr(psi))
    if rc:
        raise ValueError("invalid gate %d" % (-1 - rc))
    return psi


def probs(psi: np.ndarray) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    p = np.empty(psi.size, dtype=np.float64)
    if psi.dtype == np.complex64:
        lib().orc_probs_c64(n, _ptr(np.ascontiguousarray(psi)), _ptr(p))
    else:
        lib().orc_probs(n, _ptr(np.ascontiguousarray(psi, dtype=np.complex128)), _ptr(p))
    return p


STAT_NAMES = ["norm", "entropy", "unif_ce"] + ["M%d" % k for k in range(1, 11)] + ["zero_count"]


def stats(p: np.ndarray) -> dict:
    n = int(p.size).bit_length() - 1
    out = np.zeros(14)
    lib().orc_stats(n, _ptr(np.ascontiguousarray(p, dtype=np.float64)), _ptr(out))
    d = dict(zip(STAT_NAMES, out.tolist()))
    d["zero_count"] = int(d["zero_count"])
    d["moments"] = np.array(out[3:13])
    return d


def cycle_stats(circ) -> list:
    """Statistics after every cycle (Sec. IV: the output distribution is
    measured after each cycle t): for t = 0..D, the gates of cycles 0..t
    applied to |0..0> in list order, then stats() of the probabilities.
    Gates must be listed in nondecreasing cycle order."""
    cyc = np.asarray(circ.gates["cycle"])
    if cyc.size and (np.diff(cyc) < 0).any():
        raise ValueError("gate cycles must be nondecreasing")
    D = int(cyc.max()) if cyc.size else 0
    psi = zero_state(circ.n)
    out = []
    first = 0
    for t in range(D + 1):
        last = first + int((cyc == t).sum())
        apply_circuit(circ, psi, first, last)
        out.append(stats(probs(psi)))
        first = last
    return out


def splitmix64(seed: int, i: int) -> int:
    return int(lib().orc_splitmix64(seed, i))


def sample_from_words(p: np.ndarray, words: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    words = np.ascontiguousarray(words, dtype=np.uint64)
    out = np.zeros(words.size, dtype=np.uint64)
    rc = lib().orc_sample_from_words(p.size, _ptr(p), _ptr(words), words.size, _ptr(out))
    if rc:
        raise ValueError("sampler rejected the distribution (%d)" % rc)
    return out


def sample(p: np.ndarray, k: int, seed: int) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(k, dtype=np.uint64)
    rc = lib().orc_sample(p.size, _ptr(p), seed, k, _ptr(out))
    if rc:
        raise ValueError("sampler rejected the distribution (%d)" % rc)
    return out


def cross_entropy(p: np.ndarray, samples: np.ndarray):
    """Returns (CE, delta_H, number of zero-probability samples)."""
    n = int(p.size).bit_length() - 1
    p = np.ascontiguousarray(p, dtype=np.float64)
    x = np.ascontiguousarray(samples, dtype=np.uint64)
    ce = ctypes.c_double()
    dh = ctypes.c_double()
    z = lib().orc_cross_entropy(n, _ptr(p), _ptr(x), x.size, ctypes.byref(ce), ctypes.byref(dh))
    if z < 0:
        raise ValueError("a sample is not an %d-bit string" % n)
    return ce.value, dh.value, int(z)


def adjoint(circ, samples: np.ndarray):
    """Returns (loss, grad) of L = -mean ln p_theta(x_i) (FP64 adjoint)."""
    g, theta, mats = _circuit_arrays(circ)
    x = np.ascontiguousarray(samples, dtype=np.uint64)
    grad = np.zeros(max(theta.size, 1))
    loss = ctypes.c_double()
    rc = lib().orc_adjoint(circ.n, _ptr(g), g.shape[0], _ptr(theta), theta.size,
                           _ptr(mats), mats.size // 8, _ptr(x), x.size,
                           ctypes.byref(loss), _ptr(grad))
    if rc:
        raise ValueError("adjoint failed (%d)" % rc)
    return loss.value, grad[:theta.size]


PAIR_NAMES = ["norm_a", "norm_b", "overlap_re", "overlap_im", "fidelity", "xent", "unif_ce",
              "delta_h", "corr", "zero_a", "zero_mass_b"]


def pair_stats(a: np.ndarray, b: np.ndarray, nbins: int = 0, zmin: float = -8.0, zmax: float = 4.0):
    """Pair statistics of the ideal output a and another output b (complex
    amplitudes of the same size): a dict of PAIR_NAMES, and for nbins > 0 the
    histogram of z = ln(N p_a) as a (3, nbins + 2) uint64 array (counts,
    integer masses of p_a and of p_b; slots nbins and nbins + 1 are below and
    above the range)."""
    assert a.shape == b.shape
    n = int(a.size).bit_length() - 1
    a = np.ascontiguousarray(a, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    out = np.zeros(11)
    hist = np.zeros(3 * (nbins + 2) if nbins > 0 else 1, dtype=np.uint64)
    rc = lib().orc_pair_stats(n, _ptr(a), _ptr(b), nbins, zmin, zmax, _ptr(out), _ptr(hist))
    if rc:
        raise ValueError("pair statistics rejected the input (%d)" % rc)
    d = dict(zip(PAIR_NAMES, out.tolist()))
    d["zero_a"] = int(d["zero_a"])
    return d, (hist.reshape(3, nbins + 2) if nbins > 0 else None)


def num_threads() -> int:
    return int(lib().orc_num_threads())
