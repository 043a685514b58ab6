"""Host-side checks of the HIP library (no GPU needed).

* every function declared in include/*.h is exported by libsv.so;
* the planner (specialisation, diagonal folding, fusion, sweep grouping,
  program encoding) replayed on the host matches the FP64 reference for
  every mode, at sizes that span several tiles;
* argument errors are reported, not crashed on.
"""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_1608_00263_amd import circuits as C
from paper_1608_00263_amd import sv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in ("sv.h", "sv_host.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert {"sv_alloc", "sv_apply_circuit", "sv_probs", "sv_sample", "sv_cross_entropy",
            "sv_moments", "sv_backward"} <= names
    out = subprocess.run(["nm", "-D", "--defined-only", sv.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sv_[a-z0-9_]+)", out))
    assert names <= exported, names - exported
    L = sv.lib()
    for n in names:
        assert getattr(L, n) is not None


MODES = [("plain", 0, 0), ("spec", 0, 0), ("regtile", 0, 0), ("regtile", 0, 2), ("regtile", 0, 6),
         ("fused", 1, 0), ("fused", 2, 0), ("fused", 3, 0), ("fused", 4, 0), ("fused", 5, 0),
         ("tiled", 2, 9), ("tiled", 3, 11), ("tiled", 4, 12), ("tiled", 5, 13),
         # narrow tiles: the matrix cores only where a tile has the columns
         # their fragments need (vector ALU otherwise)
         ("tiled", 4, 8), ("tiled", 4, 9), ("tiled", 5, 10)]


@pytest.mark.parametrize("mode,k,t", MODES)
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_plan_replay_paper_circuit(mode, k, t, dtype):
    if dtype == "c128" and t == 13:
        t = 12
    circ = C.make_circuit(3, 5, 30, seed=3)
    ref = oracle.apply_circuit(circ)
    psi0 = np.zeros(1 << circ.n, complex)
    psi0[0] = 1
    out = sv.host_emulate(circ, psi0, dtype, mode, k, t)
    tol = 1e-5 if dtype == "c64" else 1e-12
    assert np.linalg.norm(out - ref) < tol


@pytest.mark.parametrize("mode,k,t", MODES)
def test_plan_replay_random_kinds(mode, k, t):
    # every gate kind, dense U1 matrices, CZ on arbitrary pairs, start state
    # not |0..0> (no Hadamard-layer shortcut)
    circ = C.random_unitary_circuit(12, 160, seed=77)
    psi0 = C.random_state(12, 5, dtype=np.complex128)
    ref = oracle.apply_circuit(circ, psi0.copy())
    out = sv.host_emulate(circ, psi0, "c128", mode, k, t, from_zero=False)
    assert np.linalg.norm(out - ref) < 1e-12


@pytest.mark.parametrize("budget", [20, 60, 160, 400, 2000])
@pytest.mark.parametrize("dtype,tile", [("c64", 6), ("c64", 4), ("c128", 5)])
def test_plan_replay_regtile_budgets(budget, dtype, tile):
    # the register-tile grouping at sweep budgets across the allowed range
    # (greedy, look-ahead and beam groupings, whichever needs fewest sweeps)
    circ = C.make_circuit(3, 5, 30, seed=3)
    ref = oracle.apply_circuit(circ)
    psi0 = np.zeros(1 << circ.n, complex)
    psi0[0] = 1
    out = sv.host_emulate(circ, psi0, dtype, "regtile", 0, tile, budget=budget)
    tol = 1e-5 if dtype == "c64" else 1e-12
    assert np.linalg.norm(out - ref) < tol
    rnd = C.random_unitary_circuit(12, 160, seed=78)
    p0 = C.random_state(12, 6, dtype=np.complex128)
    ref = oracle.apply_circuit(rnd, p0.copy())
    out = sv.host_emulate(rnd, p0, dtype, "regtile", 0, min(tile, 6), from_zero=False, budget=budget)
    assert np.linalg.norm(out - ref) < tol


def test_plan_sweep_budget_bounds():
    circ = C.make_circuit(3, 4, 10, seed=1)
    for bad in (1, 19, 2001):
        with pytest.raises(sv.SVError) as e:
            sv.host_plan(circ, "c64", "regtile", 0, 5, budget=bad)
        assert e.value.status == sv.SV_EINVAL
    for good in (20, 2000):
        assert sv.host_plan(circ, "c64", "regtile", 0, 5, budget=good)["sweeps"] > 0


def test_plan_replay_parametrised():
    circ = C.make_circuit(3, 4, 16, seed=8, parametrise=True, theta_seed=9, theta_std=0.3)
    ref = oracle.apply_circuit(circ)
    psi0 = np.zeros(1 << circ.n, complex)
    psi0[0] = 1
    for mode in ("regtile", "fused", "tiled", "spec"):
        out = sv.host_emulate(circ, psi0, "c128", mode, 4, 0)
        assert np.linalg.norm(out - ref) < 1e-12


def test_plan_sweep_counts_30q():
    circ = C.make_circuit(5, 6, 40, seed=2)
    plain = sv.host_plan(circ, "c64", "plain")
    spec = sv.host_plan(circ, "c64", "spec")
    reg = sv.host_plan(circ, "c64", "regtile", 0, 6)
    f5 = sv.host_plan(circ, "c64", "fused", 5)
    assert plain["sweeps"] == circ.ngates == 625
    # the Hadamard layer becomes one initialisation write
    assert spec["sweeps"] == circ.ngates - circ.n + 1
    assert reg["sweeps"] < 40 and f5["sweeps"] < 120
    assert f5["mfma_sweeps"] > 0
    # without MFMA the same blocks run on the vector ALUs
    f5v = sv.host_plan(circ, "c64", "fused", 5, no_mfma=True)
    assert f5v["mfma_sweeps"] == 0 and f5v["sweeps"] == f5["sweeps"]
    assert "mfma=1" not in sv.host_plan_describe(circ, "c64", "fused", 5, no_mfma=True)
    assert abs(plain["bytes"] - sum(
        (2 if g["kind"] != C.CZ else 1) * 8 * 2 ** 30 for g in circ.gates)) < 1


def test_host_plan_rejects_bad_gates():
    circ = C.make_circuit(2, 2, 4, seed=1)
    bad = circ.gates.copy()
    bad["q0"][0] = 9
    with pytest.raises(sv.SVError) as e:
        sv.host_plan(C.Circuit(n=4, gates=bad), "c64", "regtile")
    assert e.value.status == sv.SV_EINVAL
    bad = circ.gates.copy()
    bad["kind"][0] = 99
    with pytest.raises(sv.SVError):
        sv.host_plan(C.Circuit(n=4, gates=bad), "c64", "spec")
    bad = circ.gates.copy()
    bad["param"][0] = 0            # Hadamard cannot be parametrised
    with pytest.raises(sv.SVError):
        sv.host_plan(C.Circuit(n=4, gates=bad, theta=np.zeros(1)), "c64", "spec")


# ---------------------------------------------------------------------------
# per-cycle statistics plan: probabilities at every statistics point
# ---------------------------------------------------------------------------
def oracle_cycle_probs(circ):
    cyc = circ.gates["cycle"]
    psi = oracle.zero_state(circ.n)
    out, first = [], 0
    for t in range(int(cyc.max()) + 1):
        last = first + int((cyc == t).sum())
        oracle.apply_circuit(circ, psi, first, last)
        out.append(oracle.probs(psi))
        first = last
    return out


@pytest.mark.parametrize("dtype,mode,tile", [("c128", "regtile", 0), ("c128", "regtile", 2), ("c64", "regtile", 6),
                                             ("c64", "regtile", 3), ("c128", "spec", 0), ("c128", "plain", 0)])
def test_cycle_plan_replay_paper_circuit(dtype, mode, tile):
    circ = C.make_circuit(3, 5, 24, seed=12)
    ref = oracle_cycle_probs(circ)
    probs, rows = sv.host_cycle_emulate(circ, dtype, mode, tile)
    assert rows.size == len(ref)
    tol = 1e-12 if dtype == "c128" else 2e-6
    for t, p in enumerate(ref):
        assert np.abs(probs[rows[t]] - p).sum() < tol, t
    # cycles 1..3 are diagonal: no statistics pass of their own
    assert (rows[:4] == 0).all()
    dense = {int(c) for k, c in zip(circ.gates["kind"], circ.gates["cycle"]) if k in (C.SX, C.SY)}
    if mode == "regtile":
        assert probs.shape[0] == 1 + len(dense)


def test_cycle_plan_replay_every_gate_its_own_cycle():
    # random kinds, dense U1 gates, CZ on arbitrary pairs; gate i in cycle i
    circ = C.random_unitary_circuit(11, 90, seed=13)
    ref = oracle_cycle_probs(circ)
    for mode in ("regtile", "spec"):
        probs, rows = sv.host_cycle_emulate(circ, "c128", mode, 0)
        for t, p in enumerate(ref):
            assert np.abs(probs[rows[t]] - p).sum() < 1e-12, (mode, t)


def test_cycle_plan_rejects_unordered_cycles():
    circ = C.make_circuit(2, 5, 8, seed=14)
    g = circ.gates.copy()
    g["cycle"][3], g["cycle"][-1] = g["cycle"][-1], g["cycle"][3]
    bad = C.Circuit(n=circ.n, gates=g)
    with pytest.raises(sv.SVError) as e:
        sv.host_cycle_emulate(bad, "c128", "regtile", 0)
    assert e.value.status == sv.SV_EINVAL
    with pytest.raises(ValueError):
        oracle.cycle_stats(bad)
