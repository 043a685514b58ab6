"""Stabilizer-tableau simulation of Clifford circuits (test helper).

The tableau method of Aaronson and Gottesman ("Improved simulation of
stabilizer circuits", PRA 70, 052328, 2004), written from the paper's
description: 2n generator rows (destabilizers, then stabilizers) of X/Z
bits plus a sign bit, updated by H, S and CNOT, with measurement by row
multiplication.  Used only to pin the dense simulators on the Clifford
variant of the Sec. IV circuits (T replaced by S), where every output
probability is 0 or 2^-r (Clifford circuits are efficiently simulable).
"""
from __future__ import annotations

import numpy as np

from paper_1608_00263_amd import circuits as C


class Tableau:
    def __init__(self, n: int):
        self.n = n
        self.x = np.zeros((2 * n + 1, n), dtype=np.uint8)
        self.z = np.zeros((2 * n + 1, n), dtype=np.uint8)
        self.r = np.zeros(2 * n + 1, dtype=np.uint8)
        for i in range(n):
            self.x[i, i] = 1          # destabilizer X_i
            self.z[n + i, i] = 1      # stabilizer Z_i  (state |0...0>)

    def copy(self) -> "Tableau":
        t = Tableau.__new__(Tableau)
        t.n = self.n
        t.x, t.z, t.r = self.x.copy(), self.z.copy(), self.r.copy()
        return t

    # --- gates -------------------------------------------------------
    def h(self, a):
        self.r ^= self.x[:, a] & self.z[:, a]
        self.x[:, a], self.z[:, a] = self.z[:, a].copy(), self.x[:, a].copy()

    def s(self, a):
        self.r ^= self.x[:, a] & self.z[:, a]
        self.z[:, a] ^= self.x[:, a]

    def cnot(self, a, b):
        self.r ^= self.x[:, a] & self.z[:, b] & (self.x[:, b] ^ self.z[:, a] ^ 1)
        self.x[:, b] ^= self.x[:, a]
        self.z[:, a] ^= self.z[:, b]

    # --- row product with phase tracking ------------------------------
    def _rowsum(self, h, i):
        x1, z1 = self.x[i].astype(np.int64), self.z[i].astype(np.int64)
        x2, z2 = self.x[h].astype(np.int64), self.z[h].astype(np.int64)
        g = np.where((x1 == 1) & (z1 == 1), z2 - x2,
                     np.where((x1 == 1) & (z1 == 0), z2 * (2 * x2 - 1),
                              np.where((x1 == 0) & (z1 == 1), x2 * (1 - 2 * z2), 0)))
        tot = 2 * int(self.r[h]) + 2 * int(self.r[i]) + int(g.sum())
        self.r[h] = 0 if tot % 4 == 0 else 1
        self.x[h] ^= self.x[i]
        self.z[h] ^= self.z[i]

    def measure(self, a, forced=None):
        """Measure qubit a.  Returns (outcome, probability of it)."""
        n = self.n
        rows = np.nonzero(self.x[n:2 * n, a])[0]
        if rows.size:
            p = n + int(rows[0])
            for i in range(2 * n):
                if i != p and self.x[i, a]:
                    self._rowsum(i, p)
            self.x[p - n], self.z[p - n], self.r[p - n] = self.x[p], self.z[p], self.r[p]
            self.x[p] = 0
            self.z[p] = 0
            self.z[p, a] = 1
            out = 0 if forced is None else int(forced)
            self.r[p] = out
            return out, 0.5
        s = 2 * n
        self.x[s] = 0
        self.z[s] = 0
        self.r[s] = 0
        for i in range(n):
            if self.x[i, a]:
                self._rowsum(s, i + n)
        return int(self.r[s]), 1.0

    def probability(self, bits) -> float:
        """Probability of the basis state with bit q = bits[q]."""
        t = self.copy()
        prob = 1.0
        for a in range(self.n):
            out, pr = t.measure(a, forced=bits[a])
            if pr == 1.0 and out != bits[a]:
                return 0.0
            prob *= pr
        return prob

    def num_random(self) -> int:
        """Number r of random outcomes when measuring all qubits (p = 2^-r)."""
        t = self.copy()
        r = 0
        for a in range(self.n):
            out, pr = t.measure(a, forced=0)
            if pr < 1.0:
                r += 1
            elif out != 0:
                # deterministic 1: keep going, the count is unaffected
                pass
        return r


def run_clifford(circ) -> Tableau:
    """Simulate a circuit made only of Clifford kinds (global phases dropped)."""
    t = Tableau(circ.n)
    for g in circ.gates:
        k, a, b = int(g["kind"]), int(g["q0"]), int(g["q1"])
        if int(g["param"]) >= 0:
            raise ValueError("parametrised gate in a Clifford circuit")
        if k == C.H:
            t.h(a)
        elif k == C.S:
            t.s(a)
        elif k == C.SDG:
            t.s(a); t.s(a); t.s(a)
        elif k == C.Z:
            t.s(a); t.s(a)
        elif k == C.X:
            t.h(a); t.s(a); t.s(a); t.h(a)
        elif k == C.Y:
            t.h(a); t.s(a); t.s(a); t.h(a)      # X
            t.s(a); t.s(a)                      # then Z: Y up to phase
        elif k == C.SX:                         # RX(pi/2) ~ H S H
            t.h(a); t.s(a); t.h(a)
        elif k == C.SXDG:
            t.h(a); t.s(a); t.s(a); t.s(a); t.h(a)
        elif k == C.SY:                         # RY(pi/2) = X H: H first
            t.h(a)
            t.h(a); t.s(a); t.s(a); t.h(a)
        elif k == C.SYDG:                       # H X: X first
            t.h(a); t.s(a); t.s(a); t.h(a)
            t.h(a)
        elif k == C.CZ:
            t.h(b); t.cnot(a, b); t.h(b)
        else:
            raise ValueError("non-Clifford kind %s" % C.KIND_NAMES[k])
    return t
