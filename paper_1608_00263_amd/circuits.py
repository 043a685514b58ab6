"""Seeded generator for the random 2D-lattice circuits of Sec. IV.

This module only builds *inputs*: gate records (kind, qubits, cycle,
parameter index), rotation offsets and random words.  It contains none of
the simulation arithmetic (no gate matrices, no amplitudes), so both the
HIP library and the FP64 reference implementation consume its output
without sharing any numerical code.

Circuit family (Sec. IV, the enumerated construction and the three
placement rules that follow it):

* cycle 0 is a Hadamard on every qubit;
* each of the next ``depth`` cycles places CZ gates from one of eight
  nearest-neighbour layouts (Fig. 6), taken in a fixed rotation, and then
  single-qubit gates drawn from {X^1/2, Y^1/2, T} on qubits that are idle
  in the current cycle, subject to the rules:
  - a qubit gets a single-qubit gate only if it was part of a CZ in the
    previous cycle;
  - its first single-qubit gate after the Hadamard is T;
  - otherwise the gate differs from the last single-qubit gate on it;
* no final Hadamard layer (Sec. IV, the paragraph after the rules).

Fig. 6 itself is not available, so the eight layouts are the family
below (a reading calibrated against the "gates per level" column of
Table I):

* ``H_a`` (a = 0..3): CZ on ((r, c), (r, c+1)) for every row r and every
  column c with c + 1 < C and c = a + 2r (mod 4);
* ``V_a`` (a = 0..3): CZ on ((r, c), (r+1, c)) for every column c and
  every row r with r + 1 < R and r = a + 2c (mod 4);
* cycle t >= 1 uses ``LAYOUT_ORDER[(t - 1) % 8]``.

Qubit q = r * C + c is bit q of an amplitude index.  Random choices use
SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) written out here from its
published definition.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --- gate-record format -------------------------------------------------
# The numeric codes are an interchange format (the same values appear in
# the C header of the library and in the reference implementation).
H, CZ, T, SX, SY, S, X, Y, Z, TDG, SDG, SXDG, SYDG, U1 = range(14)
KIND_NAMES = ["H", "CZ", "T", "SX", "SY", "S", "X", "Y", "Z",
              "TDG", "SDG", "SXDG", "SYDG", "U1"]
# kinds that may carry a rotation offset (angle = nominal + theta[param]);
# the inverse kinds are included so that an inverted parametrised circuit
# stays expressible (the rotation R(a) is inverted by R(-a)).
PARAMETRISABLE = (T, SX, SY, TDG, SXDG, SYDG)
# inverse of each fixed kind (U1 handled separately, CZ/H/X/Y/Z self-inverse)
INVERSE = {H: H, CZ: CZ, T: TDG, SX: SXDG, SY: SYDG, S: SDG, X: X, Y: Y,
           Z: Z, TDG: T, SDG: S, SXDG: SX, SYDG: SY}

GATE_DTYPE = np.dtype([("kind", "<i4"), ("q0", "<i4"), ("q1", "<i4"),
                       ("cycle", "<i4"), ("param", "<i4"), ("mat", "<i4")])

# Layout rotation (see module docstring).  Each entry is (orientation, a).
LAYOUT_ORDER: Tuple[Tuple[str, int], ...] = (
    ("H", 0), ("H", 2), ("V", 0), ("V", 1),
    ("V", 3), ("V", 2), ("H", 1), ("H", 3))

MASK64 = (1 << 64) - 1
GAMMA64 = 0x9E3779B97F4A7C15


def splitmix64_mix(z: int) -> int:
    """SplitMix64 output function applied to a 64-bit state value."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class SplitMix64:
    """Sequential SplitMix64 stream: state += gamma, then mix."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + GAMMA64) & MASK64
        return splitmix64_mix(self.state)

    def below(self, k: int) -> int:
        """Uniform integer in [0, k) by the multiply-high method (Lemire)."""
        return (self.next() * k) >> 64

    def unit(self) -> float:
        """Uniform double in [0, 1) with 53 random bits."""
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)


def splitmix64_words(seed: int, count: int) -> np.ndarray:
    """The first ``count`` outputs of SplitMix64 from ``seed`` (uint64)."""
    g = SplitMix64(seed)
    return np.array([g.next() for _ in range(count)], dtype=np.uint64)


def layout_pairs(rows: int, cols: int, orient: str, a: int) -> List[Tuple[int, int]]:
    """CZ pairs (q_low, q_high) of one layout, in a fixed order."""
    out = []
    if orient == "H":
        for r in range(rows):
            for c in range(cols - 1):
                if (c - a - 2 * r) % 4 == 0:
                    out.append((r * cols + c, r * cols + c + 1))
    else:
        for c in range(cols):
            for r in range(rows - 1):
                if (r - a - 2 * c) % 4 == 0:
                    out.append((r * cols + c, (r + 1) * cols + c))
    out.sort()
    return out


@dataclasses.dataclass
class Circuit:
    """A gate list plus the data some kinds refer to.

    ``gates`` is a structured array with fields kind, q0, q1 (-1 for
    single-qubit gates), cycle, param (-1 or index into ``theta``) and
    mat (-1 or index into ``mats``, used by U1 only).
    """
    n: int
    gates: np.ndarray
    theta: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))
    mats: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros((0, 2, 2), dtype=np.complex128))
    rows: int = 0
    cols: int = 0
    depth: int = 0

    @property
    def ngates(self) -> int:
        return int(self.gates.shape[0])

    @property
    def nparams(self) -> int:
        return int(self.theta.shape[0])

    def counts(self) -> dict:
        k = self.gates["kind"]
        return {name: int((k == i).sum()) for i, name in enumerate(KIND_NAMES)
                if (k == i).any()}

    def gates_per_level(self) -> float:
        """Gates per clock cycle, counting the Hadamard layer (Table I)."""
        return self.ngates / self.depth

    def with_theta(self, theta: np.ndarray) -> "Circuit":
        return dataclasses.replace(self, theta=np.asarray(theta, dtype=np.float64).copy())

    def prefix_cycles(self, last_cycle: int) -> "Circuit":
        """Gates of cycles 0..last_cycle (same parameters)."""
        keep = self.gates["cycle"] <= last_cycle
        return dataclasses.replace(self, gates=self.gates[keep].copy(),
                                   depth=min(self.depth, last_cycle))

    def inverse(self) -> "Circuit":
        """The adjoint circuit (gates reversed and inverted).

        Parametrised gates keep their parameter index: R(nominal + theta)
        is inverted by the inverse kind, whose nominal angle is negated,
        together with the negated offset, R(-nominal - theta).
        """
        g = self.gates[::-1].copy()
        mats = self.mats.copy()
        for i in range(g.shape[0]):
            k = int(g["kind"][i])
            if k == U1:
                mats[g["mat"][i]] = self.mats[g["mat"][i]].conj().T
            else:
                g["kind"][i] = INVERSE[k]
        return dataclasses.replace(self, gates=g, mats=mats, theta=-self.theta)


def make_gates(records: Sequence[Tuple[int, int, int, int, int, int]]) -> np.ndarray:
    arr = np.zeros(len(records), dtype=GATE_DTYPE)
    for i, r in enumerate(records):
        arr[i] = r
    return arr


def make_circuit(rows: int, cols: int, depth: int, seed: int,
                 rules: str = "paper", clifford: bool = False,
                 parametrise: bool = False, theta_seed: Optional[int] = None,
                 theta_std: float = 0.05) -> Circuit:
    """Build one random circuit of the Sec. IV family.

    rules       "paper" (the three placement rules) or "all_idle" (every
                qubit that is not in a CZ in this cycle gets a uniform draw
                from the three gates).
    clifford    replace T by S = diag(1, i) (a Clifford circuit, used for
                exact checks at any size).
    parametrise give every non-Hadamard single-qubit gate its own rotation
                offset theta_g ~ N(0, theta_std^2) (Box-Muller from a
                SplitMix64 stream seeded with ``theta_seed``).
    """
    if rows < 1 or cols < 1 or depth < 0:
        raise ValueError("bad grid or depth")
    n = rows * cols
    rng = SplitMix64(seed)
    recs: List[Tuple[int, int, int, int, int, int]] = []
    for q in range(n):
        recs.append((H, q, -1, 0, -1, -1))
    last_1q = [-1] * n          # last single-qubit gate kind (after cycle 0)
    prev_busy = [False] * n     # in a CZ during the previous cycle
    tkind = S if clifford else T
    nparam = 0
    for t in range(1, depth + 1):
        orient, a = LAYOUT_ORDER[(t - 1) % 8]
        pairs = layout_pairs(rows, cols, orient, a)
        busy = [False] * n
        for (qa, qb) in pairs:
            recs.append((CZ, qa, qb, t, -1, -1))
            busy[qa] = busy[qb] = True
        for q in range(n):
            if busy[q]:
                continue
            if rules == "paper":
                if not prev_busy[q]:
                    continue
                if last_1q[q] < 0:
                    kind = tkind
                else:
                    options = [k for k in (tkind, SX, SY) if k != last_1q[q]]
                    kind = options[rng.next() >> 63]
            elif rules == "all_idle":
                kind = (tkind, SX, SY)[rng.below(3)]
            else:
                raise ValueError("rules must be 'paper' or 'all_idle'")
            p = -1
            if parametrise:
                p = nparam
                nparam += 1
            recs.append((kind, q, -1, t, p, -1))
            last_1q[q] = kind
        prev_busy = busy
    theta = np.zeros(nparam, dtype=np.float64)
    if parametrise and nparam:
        theta = normal_draws(theta_seed if theta_seed is not None else seed + 1,
                             nparam) * theta_std
    return Circuit(n=n, gates=make_gates(recs), theta=theta, rows=rows,
                   cols=cols, depth=depth)


# Denser family of App. E: every qubit takes part in exactly one CZ per
# layer, with periodic boundary conditions.  The four perfect matchings of
# nearest-neighbour bonds on the R x C torus (horizontal or vertical, bonds
# starting at even or odd columns / rows) are taken in this rotation, so
# every bond is used once per four layers (R, C >= 4).
DENSE_LAYOUT_ORDER: Tuple[Tuple[str, int], ...] = (("H", 0), ("V", 0), ("H", 1), ("V", 1))


def dense_layout_pairs(rows: int, cols: int, orient: str, a: int) -> List[Tuple[int, int]]:
    """CZ pairs (q_low, q_high) of one periodic perfect-matching layout."""
    out = []
    if orient == "H":
        for r in range(rows):
            for c in range(a, cols, 2):
                q0, q1 = r * cols + c, r * cols + (c + 1) % cols
                out.append((min(q0, q1), max(q0, q1)))
    else:
        for c in range(cols):
            for r in range(a, rows, 2):
                q0, q1 = r * cols + c, ((r + 1) % rows) * cols + c
                out.append((min(q0, q1), max(q0, q1)))
    out.sort()
    return out


def make_dense_periodic_circuit(rows: int, cols: int, layers: int, seed: int,
                                clifford: bool = False) -> Circuit:
    """One random circuit of the denser family of App. E.

    Cycle 0 is a Hadamard on every qubit.  Layer l = 1..layers is a cycle
    of single-qubit gates on every qubit followed by a cycle of CZ gates in
    which every qubit takes part in exactly one CZ (layout
    DENSE_LAYOUT_ORDER[(l - 1) % 4], periodic boundaries).  The single-qubit
    gates follow the placement rules of Sec. IV that apply here: the first
    one on a qubit is T, each later one is drawn uniformly from {T, X^1/2,
    Y^1/2} minus the previous one on that qubit.  Every gate of layer l has
    cycle l, so statistics after each cycle are per layer, as depth is
    counted in App. E.  rows and cols must be even (a perfect matching of
    the torus in both orientations).
    """
    if rows < 2 or cols < 2 or rows % 2 or cols % 2 or layers < 0:
        raise ValueError("the dense periodic family needs even rows and cols >= 2")
    n = rows * cols
    rng = SplitMix64(seed)
    recs: List[Tuple[int, int, int, int, int, int]] = [(H, q, -1, 0, -1, -1) for q in range(n)]
    tkind = S if clifford else T
    last_1q = [-1] * n
    for l in range(1, layers + 1):
        for q in range(n):
            if last_1q[q] < 0:
                kind = tkind
            else:
                options = [k for k in (tkind, SX, SY) if k != last_1q[q]]
                kind = options[rng.next() >> 63]
            recs.append((kind, q, -1, l, -1, -1))
            last_1q[q] = kind
        orient, a = DENSE_LAYOUT_ORDER[(l - 1) % 4]
        for (qa, qb) in dense_layout_pairs(rows, cols, orient, a):
            recs.append((CZ, qa, qb, l, -1, -1))
    return Circuit(n=n, gates=make_gates(recs), rows=rows, cols=cols, depth=layers)


# --- errors (Sec. III and App. D) ----------------------------------------
PAULIS = (X, Y, Z)
# the 15 non-identity two-qubit Paulis (first qubit, second qubit), -1 = I
PAULI_PAIRS: Tuple[Tuple[int, int], ...] = tuple(
    (a, b) for a in (-1, X, Y, Z) for b in (-1, X, Y, Z) if not (a == -1 and b == -1))


def error_counts(circ: Circuit) -> Tuple[int, int]:
    """(g1, g2): the one-qubit gates (the Hadamard layer included) and the
    two-qubit gates of a circuit, the counts of Eq. (6)."""
    k = circ.gates["kind"]
    g2 = int((k == CZ).sum())
    return int(k.size) - g2, g2


def noisy_trajectory(circ: Circuit, r1: float, r2: float, r_init: float, r_mes: float,
                     seed: int) -> Tuple[Circuit, int]:
    """One Monte Carlo trajectory of the depolarizing error model of Sec. III
    (the simulations behind Figs. 4 and 5): after each one-qubit gate, with
    probability r1, one of X, Y, Z (r1 / 3 each); after each CZ, with
    probability r2, one of the 15 non-identity two-qubit Paulis (r2 / 15
    each); a bit flip of each qubit's initial |0> with probability r_init,
    written as Z after its cycle-0 Hadamard (H X = Z H); a bit flip before
    each measurement with probability r_mes, an X after the last gate.
    Inserted gates carry the cycle of the gate they follow.  Returns the
    trajectory and the number of inserted Paulis.  The Hadamard layer counts
    as one-qubit gates.  All draws come from a SplitMix64 stream."""
    g = SplitMix64(seed)
    n = circ.n
    recs: List[Tuple[int, int, int, int, int, int]] = []
    inserted = 0
    first_h = [True] * n
    last_cycle = int(circ.gates["cycle"].max()) if circ.ngates else 0
    for rec in circ.gates:
        kind, q0, q1, cyc = int(rec["kind"]), int(rec["q0"]), int(rec["q1"]), int(rec["cycle"])
        recs.append(tuple(int(v) for v in rec))
        if kind == CZ:
            if g.unit() < r2:
                pa, pb = PAULI_PAIRS[g.below(15)]
                for pk, q in ((pa, q0), (pb, q1)):
                    if pk >= 0:
                        recs.append((pk, q, -1, cyc, -1, -1))
                        inserted += 1
            continue
        if kind == H and cyc == 0 and first_h[q0]:
            first_h[q0] = False
            if g.unit() < r_init:
                recs.append((Z, q0, -1, 0, -1, -1))
                inserted += 1
        if g.unit() < r1:
            recs.append((PAULIS[g.below(3)], q0, -1, cyc, -1, -1))
            inserted += 1
    for q in range(n):
        if g.unit() < r_mes:
            recs.append((X, q, -1, last_cycle, -1, -1))
            inserted += 1
    out = dataclasses.replace(circ, gates=make_gates(recs))
    return out, inserted


def single_error_circuit(circ: Circuit, qubit: int, cycle: int, kind: int) -> Circuit:
    """The circuit with one Pauli error (X, a bit flip, or Z, a phase flip)
    on ``qubit`` at the end of ``cycle`` (App. D: an ideal circuit against
    the same circuit with a single error at one location)."""
    if kind not in (X, Y, Z):
        raise ValueError("a single error is a Pauli X, Y or Z")
    cyc = circ.gates["cycle"]
    if not (0 <= qubit < circ.n) or cycle < 0 or cycle > int(cyc.max()):
        raise ValueError("no such location")
    at = int(np.searchsorted(cyc, cycle, side="right"))   # after the last gate of the cycle
    err = np.zeros(1, dtype=GATE_DTYPE)
    err[0] = (kind, qubit, -1, cycle, -1, -1)
    gates = np.concatenate([circ.gates[:at], err, circ.gates[at:]])
    return dataclasses.replace(circ, gates=gates)


def normal_draws(seed: int, count: int) -> np.ndarray:
    """Standard normal deviates by the Box-Muller transform."""
    g = SplitMix64(seed)
    out = np.empty(count, dtype=np.float64)
    i = 0
    while i < count:
        u1 = 1.0 - g.unit()          # (0, 1]
        u2 = g.unit()
        rad = math.sqrt(-2.0 * math.log(u1))
        out[i] = rad * math.cos(2.0 * math.pi * u2)
        if i + 1 < count:
            out[i + 1] = rad * math.sin(2.0 * math.pi * u2)
        i += 2
    return out


def random_unitary_circuit(n: int, ngates: int, seed: int,
                           diag_fraction: float = 0.3) -> Circuit:
    """Generic test circuit: random qubits, all kinds, random dense U1.

    The dense 2x2 matrices are Haar-random unitaries (QR of a complex
    Gaussian matrix with the phase fix of Mezzadri 2007); they are
    inputs, drawn here so that both implementations see the same data.
    """
    g = SplitMix64(seed)
    recs = []
    mats = []
    fixed = [H, T, SX, SY, S, X, Y, Z, TDG, SDG, SXDG, SYDG]
    for i in range(ngates):
        u = g.unit()
        if n >= 2 and u < diag_fraction:
            a = g.below(n)
            b = g.below(n - 1)
            b = b + 1 if b >= a else b
            recs.append((CZ, min(a, b), max(a, b), i, -1, -1))
        elif u < diag_fraction + 0.25:
            q = g.below(n)
            z = np.array([normal_draws(g.next(), 8)]).reshape(2, 2, 2)
            m = z[..., 0] + 1j * z[..., 1]
            qm, rm = np.linalg.qr(m)
            d = np.diag(rm)
            qm = qm * (d / np.abs(d))
            recs.append((U1, q, -1, i, -1, len(mats)))
            mats.append(qm)
        else:
            q = g.below(n)
            recs.append((fixed[g.below(len(fixed))], q, -1, i, -1, -1))
    mats_arr = np.array(mats, dtype=np.complex128).reshape(-1, 2, 2)
    return Circuit(n=n, gates=make_gates(recs), mats=mats_arr, depth=ngates)


def random_state(n: int, seed: int, dtype=np.complex64, normalise: bool = True) -> np.ndarray:
    """Seeded complex Gaussian amplitudes (a synthetic Porter-Thomas state)."""
    rs = np.random.Generator(np.random.PCG64(seed))
    z = rs.standard_normal(2 << n).view(np.complex128)
    if normalise:
        z /= np.sqrt(np.vdot(z, z).real)
    return z.astype(dtype)


def random_probabilities(N: int, seed: int, zeros: int = 0) -> np.ndarray:
    """Seeded Dirichlet(1,...,1) probability vector, optional exact zeros."""
    rs = np.random.Generator(np.random.PCG64(seed))
    p = rs.exponential(size=N)
    if zeros:
        p[rs.choice(N, size=min(zeros, N - 1), replace=False)] = 0.0
    return p / p.sum()


ENSEMBLE_GRIDS: Tuple[Tuple[int, int], ...] = ((4, 5), (4, 6), (5, 5))


def make_ensemble(count: int, meta_seed: int = 3, grids: Sequence[Tuple[int, int]] = ENSEMBLE_GRIDS,
                  depth_range: Tuple[int, int] = (20, 40), seed0: int = 3000) -> List[Circuit]:
    """Ensemble of Sec. IV circuits of uneven size and depth: instance i has a
    grid drawn uniformly from ``grids`` and a depth drawn uniformly from
    ``depth_range`` (inclusive) by a SplitMix64 stream seeded with
    ``meta_seed``, and circuit seed ``seed0 + i``."""
    g = SplitMix64(meta_seed)
    lo, hi = depth_range
    out = []
    for i in range(count):
        r, c = grids[g.below(len(grids))]
        d = lo + g.below(hi - lo + 1)
        out.append(make_circuit(r, c, d, seed=seed0 + i))
    return out
