"""Full-size GPU checks.

The benchmark's own workload, the 30-qubit depth-40 circuit of the 5x6 grid
in complex64 with register tiles of 6 qubits (the launch configuration the
benchmark times), is checked against two other computations of the same
state on the GPU: complex128 per-gate sweeps (a different kernel family and
precision) and complex128 register tiles; and its Clifford variant against a
stabilizer tableau.

The 35-qubit, depth-40 circuit of the 5x7 grid in complex64 (a 256 GiB
state) is checked through properties that hold at any size, since no
reference can hold the state:

* the Clifford variant (T replaced by S) against a stabilizer tableau: the
  probability of every sampled bit string is exactly 2^-r, the entropy is
  r ln 2 and 2^n - 2^r outcomes have probability zero;
* the circuit followed by its inverse returns |0...0>;
* the output of the circuit itself approaches Porter-Thomas (Sec. IV): the
  statistics after every cycle never exceed the Porter-Thomas entropy by
  4 sigma (an error would), come within 4 sigma of it in cycles 30..40, and
  10^6 samples drawn from the output have cross entropy equal to its entropy
  (Delta H = 1 up to the sample error).

The 30-qubit prefix of the 35-qubit family (5x6 grid, the same seed) is
compared with the FP64 reference directly (about a minute of host time).
"""
import math

import numpy as np
import pytest

from paper_1608_00263_amd import circuits as C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_00263_amd import sv  # noqa: E402

EULER_GAMMA = 0.5772156649015329
N35_BYTES = 8 * 2 ** 35


def _free_bytes():
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info(0)
    return free


@pytest.fixture(scope="module")
def st35():
    if _free_bytes() < N35_BYTES + (4 << 30):
        pytest.skip("a 35-qubit complex64 state needs 260 GiB of free device memory")
    print("allocating the 35-qubit state", flush=True)
    st = sv.State(35, "c64")
    yield st
    st.close()
    del st
    torch.cuda.empty_cache()


@pytest.fixture
def st30():
    # per test, so that nothing of it is held when the 35-qubit state needs
    # all but a few GiB of the device
    print("allocating the 30-qubit state", flush=True)
    st = sv.State(30, "c64")
    yield st
    st.close()
    del st
    torch.cuda.empty_cache()


def _check_clifford(st, circ, n, nsamp, seed):
    from tests.stabilizer import run_clifford
    m = st.moments()
    tab = run_clifford(circ)
    r = tab.num_random()
    assert abs(m["norm"] - 1.0) < 1e-5
    assert abs(m["entropy"] - r * math.log(2.0)) < 1e-4
    assert m["zero_count"] == 2 ** n - 2 ** r
    xs = st.sample(nsamp, seed)
    for x in xs:
        bits = [(int(x) >> q) & 1 for q in range(n)]
        want = tab.probability(bits)
        got = float(st.probs(int(x), 1).cpu()[0])
        assert want == 2.0 ** -r
        assert abs(got / want - 1.0) < 1e-4, (int(x), got, want)


def test_c2_clifford_variant_vs_tableau(st30):
    circ = C.make_circuit(5, 6, 40, seed=2, clifford=True)
    st30.apply(circ, "regtile", 0, 6, from_zero=True)
    _check_clifford(st30, circ, 30, 64, 78)


def _check_clifford_cycles(st, circ, n):
    # statistics after every cycle against the tableau of each cycle prefix:
    # uniform on 2^r_t outcomes, entropy r_t ln 2, M_k = 2^{(n - r_t)(k - 1)}
    from tests.stabilizer import run_clifford
    got = st.cycle_moments(circ, "regtile", 6)
    assert len(got) == circ.depth + 1
    for t, m in enumerate(got):
        r = run_clifford(circ.prefix_cycles(t)).num_random()
        assert abs(m["entropy"] - r * math.log(2.0)) < 1e-4, (t, m["entropy"], r)
        assert abs(m["M2"] / 2.0 ** (n - r) - 1.0) < 1e-4, t
        assert abs(m["norm"] - 1.0) < 1e-5, t
    print("clifford cycles: r from %d to %d" % (round(got[4]["entropy"] / math.log(2)),
                                               round(got[-1]["entropy"] / math.log(2))), flush=True)


def test_c2_clifford_cycles_vs_tableau(st30):
    _check_clifford_cycles(st30, C.make_circuit(5, 6, 40, seed=2, clifford=True), 30)


def test_c2_register_tiles_vs_per_gate_c128(st30):
    circ = C.make_circuit(5, 6, 40, seed=2)
    print("30 qubits: complex64 register tiles", flush=True)
    st30.apply(circ, "regtile", 0, 6, from_zero=True)
    m64 = st30.moments()
    xs = st30.sample(10 ** 5, 1002)
    ce64, dh64, _ = st30.cross_entropy(xs, norm=m64["norm"])
    print("30 qubits: complex128 per-gate sweeps", flush=True)
    ref = sv.State(30, "c128")
    ref.apply(circ, "plain", from_zero=True)
    d = float(torch.linalg.vector_norm(st30.tensor.to(torch.complex128) - ref.tensor))
    assert d <= 1e-4, d
    m128 = ref.moments()
    assert abs(m64["entropy"] - m128["entropy"]) <= 1e-4
    assert abs(m64["unif_ce"] - m128["unif_ce"]) <= 1e-4
    np.testing.assert_allclose(m64["moments"], m128["moments"], rtol=1e-3)
    ce128, dh128, _ = ref.cross_entropy(xs)
    assert abs(ce64 - ce128) <= 1e-4 and abs(dh64 - dh128) <= 1e-4
    print("30 qubits: complex128 register tiles", flush=True)
    rt = sv.State(30, "c128")
    rt.apply(circ, "regtile", 0, 5, from_zero=True)
    d128 = float(torch.linalg.vector_norm(rt.tensor - ref.tensor))
    assert d128 <= 1e-11, d128
    rt.close()
    ref.close()
    del rt, ref
    torch.cuda.empty_cache()


def test_c2_shape_seed5_vs_reference_30q():
    # the 35-qubit run's 30-qubit prefix (the same generator and seed on the
    # 5x6 grid) against the FP64 reference: complex64 in the benchmark's
    # launch configuration (register tiles of 6 qubits) and as the autotuner
    # picks it, complex128 register tiles and per-gate sweeps, and the cross
    # entropy of 10^5 samples of the complex64 state
    import oracle
    circ = C.make_circuit(5, 6, 40, seed=5)
    print("reference run, 30 qubits complex128 (%d host threads)" % oracle.num_threads(), flush=True)
    ref = oracle.apply_circuit(circ)
    pref = oracle.probs(ref)
    dref = torch.from_numpy(ref).to("cuda")
    del ref
    st = sv.State(30, "c64")
    for mode, t in (("regtile", 6), ("auto", 0)):
        st.apply(circ, mode, 0, t, from_zero=True)
        d = float(torch.linalg.vector_norm(st.tensor.to(torch.complex128) - dref))
        print("30 qubits complex64 %s: |psi - psi_ref| = %.3e" % (mode, d), flush=True)
        assert d <= 1e-4, (mode, d)
    m = st.moments()
    xs = st.sample(10 ** 5, 1005)
    ce, dh, z = st.cross_entropy(xs, norm=m["norm"])
    ce0, dh0, z0 = oracle.cross_entropy(pref, xs)
    print("30 qubits complex64: ce %.9f vs %.9f" % (ce, ce0), flush=True)
    assert z == z0 == 0 and abs(ce - ce0) <= 1e-4 and abs(dh - dh0) <= 1e-4
    want = oracle.stats(pref)
    assert abs(m["entropy"] - want["entropy"]) <= 1e-4 and abs(m["unif_ce"] - want["unif_ce"]) <= 1e-4
    st.close()
    del st, pref
    torch.cuda.empty_cache()
    s128 = sv.State(30, "c128")
    for mode, t in (("regtile", 5), ("plain", 0)):
        s128.apply(circ, mode, 0, t, from_zero=True)
        d = float(torch.linalg.vector_norm(s128.tensor - dref))
        print("30 qubits complex128 %s: |psi - psi_ref| = %.3e" % (mode, d), flush=True)
        assert d <= 1e-11, (mode, d)
    s128.close()
    del s128, dref
    torch.cuda.empty_cache()


def test_c3_full_ensemble_subset():
    # the 512-instance ensemble of the benchmark (67 GB of complex64 states)
    # in one call; every 16th instance against a single-state run of the same
    # circuit, and its 20-qubit ones against the FP64 reference
    import oracle
    circs = C.make_ensemble(512)
    print("ensemble: allocating 512 states", flush=True)
    states = [sv.State(c.n, "c64") for c in circs]
    res = sv.apply_batch(states, circs)
    one = {}
    for i in range(0, 512, 16):
        c = circs[i]
        ref_gpu = sv.State(c.n, "c64")
        ref_gpu.apply(c, "regtile", from_zero=True)
        d = float(torch.linalg.vector_norm(states[i].tensor - ref_gpu.tensor))
        assert d <= 1e-5, (i, d)
        m = ref_gpu.moments()
        assert abs(res[i]["entropy"] - m["entropy"]) < 1e-6, i
        np.testing.assert_allclose(res[i]["moments"][:5], m["moments"][:5], rtol=1e-5)
        ref_gpu.close()
        if c.n == 20:
            print("ensemble instance %d: FP64 reference" % i, flush=True)
            ref = oracle.apply_circuit(c)
            assert np.linalg.norm(states[i].amplitudes() - ref) <= 1e-4, i
            want = oracle.stats(oracle.probs(ref))
            assert abs(res[i]["entropy"] - want["entropy"]) < 1e-4, i
            one[i] = True
    assert len(one) == 9
    for st in states:
        st.close()
    del states
    torch.cuda.empty_cache()


def test_c4_adjoint_full_size():
    # the benchmark's gradient workload (5x5 grid, 25 qubits, depth 30, 216
    # parameters, 10^4 samples of the theta = 0 circuit): the complex64
    # adjoint against the complex128 one over every parameter, and the
    # complex128 one against central differences of the loss on 16 seeded
    # parameters (h = 1e-4: truncation near 1e-8, rounding near 1e-10)
    circ = C.make_circuit(5, 5, 30, seed=4, parametrise=True, theta_seed=4004, theta_std=0.05)
    st = sv.State(25, "c64")
    st.apply(circ.with_theta(np.zeros(circ.nparams)), "regtile", 0, 6, from_zero=True)
    xs = st.sample(10 ** 4, 1004)
    loss64, g64 = st.backward(circ, xs)
    st.close()
    s128 = sv.State(25, "c128")
    loss128, g128 = s128.backward(circ, xs)
    print("C4 gradients: |g| = %.4e, max |g64 - g128| = %.3e, |g64 - g128| / |g128| = %.3e, loss diff %.2e"
          % (np.linalg.norm(g128), np.abs(g64 - g128).max(), np.linalg.norm(g64 - g128) / np.linalg.norm(g128),
             abs(loss64 - loss128)), flush=True)
    assert abs(loss64 - loss128) < 1e-4
    assert np.abs(g64 - g128).max() < 1e-4
    assert np.linalg.norm(g64 - g128) <= 1e-3 * np.linalg.norm(g128)
    h = 1e-4
    for g in np.random.default_rng(16).choice(circ.nparams, 16, replace=False):
        vals = []
        for sgn in (1.0, -1.0):
            th = circ.theta.copy()
            th[g] += sgn * h
            s128.apply(circ.with_theta(th), "regtile", 0, 5, from_zero=True)
            vals.append(s128.cross_entropy(xs)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g128[g]) < 1e-6 * max(1.0, abs(g128[g])), (int(g), fd, g128[g])
    s128.close()
    torch.cuda.empty_cache()


def test_c5_clifford_variant_vs_tableau(st35):
    circ = C.make_circuit(5, 7, 40, seed=5, clifford=True)
    print("clifford variant: %d gates" % circ.ngates, flush=True)
    st35.apply(circ, "regtile", 0, 6, from_zero=True)
    _check_clifford(st35, circ, 35, 64, 77)


def test_c5_clifford_cycles_vs_tableau(st35):
    _check_clifford_cycles(st35, C.make_circuit(5, 7, 40, seed=5, clifford=True), 35)


def test_c5_circuit_then_inverse_is_identity(st35):
    circ = C.make_circuit(5, 7, 40, seed=5)
    st35.apply(circ, "regtile", 0, 6, from_zero=True)
    st35.apply(circ.inverse(), "regtile", 0, 6)
    p0 = float(st35.probs(0, 1).cpu()[0])
    m = st35.moments()
    assert abs(m["norm"] - 1.0) < 1e-5
    assert p0 > 1.0 - 1e-4


def test_c5_auto_explores_on_the_callers_calls(st35):
    # a 256 GiB state leaves no room for a scratch copy, so the autotuner
    # times its candidates on the caller's own calls, one per call; the four
    # register-tile candidates are run, the fused ones (12 and 8 s at the
    # HBM peak against about 2 s measured) are skipped; every call leaves
    # the circuit's output state
    circ = C.make_circuit(5, 7, 40, seed=5)
    st35.apply(circ, "regtile", 0, 6, from_zero=True)
    ref = st35.moments()
    calls = 0
    while True:
        choice = st35.autotune(circ, from_zero=True)
        if choice[3]:
            break
        st35.apply(circ, "auto", from_zero=True)
        calls += 1
        m = st35.moments()
        print("auto call %d (%s tile %d budget %d): entropy %.9f" % (calls, choice[0], choice[2], choice[4],
                                                                   m["entropy"]), flush=True)
        assert abs(m["entropy"] - ref["entropy"]) < 1e-4 and abs(m["norm"] - 1.0) < 1e-5
        assert calls <= 6
    assert calls == 4 and choice[0] == "regtile", (calls, choice)
    st35.apply(circ, "auto", from_zero=True)
    m = st35.moments()
    assert abs(m["entropy"] - ref["entropy"]) < 1e-4 and abs(m["norm"] - 1.0) < 1e-5


def test_c5_porter_thomas_and_sample_cross_entropy(st35):
    # Statistics after every cycle.  sigma_H = 0.5385 2^{-n/2} nats is the
    # spread of the entropy of Porter-Thomas (Dirichlet) vectors.  An error
    # of the simulation mixes in the uniform distribution and raises the
    # entropy above the Porter-Thomas value, so no cycle from 20 on may
    # exceed it by 4 sigma; the approach from below is the circuit's own (the
    # same per-cycle deficits appear in complex64 and complex128 at 30
    # qubits), and some cycle in 30..40 must come within 4 sigma.
    circ = C.make_circuit(5, 7, 40, seed=5)
    n = 35
    N = 2.0 ** n
    hpt = n * math.log(2.0) - 1.0 + EULER_GAMMA
    sig = 0.5385 * 2.0 ** (-n / 2)
    ms = st35.cycle_moments(circ, "regtile", 6)
    deficit = [(hpt - m["entropy"]) / sig for m in ms]
    print("35 qubits: entropy deficit / sigma, cycles 30..40: %s"
          % " ".join("%.1f" % d for d in deficit[30:]), flush=True)
    assert min(deficit[20:]) > -4.0
    best = min(range(30, 41), key=lambda t: abs(deficit[t]))
    assert abs(deficit[best]) < 4.0, best
    m2_sd = math.sqrt((math.factorial(4) - 4.0) / N)
    assert abs(ms[best]["M2"] - 2.0) < 4 * m2_sd, (best, ms[best]["M2"])
    m = ms[-1]
    assert abs(m["norm"] - 1.0) < 1e-5
    for k in range(1, 6):
        assert abs(m["moments"][k - 1] / math.factorial(k) - 1.0) < 0.01 * k
    xs = st35.sample(10 ** 6, 1005)
    ce, dh, z = st35.cross_entropy(xs)
    assert z == 0
    # mean of -ln p over samples from p is the entropy, with a standard
    # error of about sqrt(pi^2/6 - 1) / sqrt(10^6) = 8.0e-4: 5 sigma
    assert abs(ce - m["entropy"]) < 4e-3
    assert abs(dh - (1.0 - (hpt - m["entropy"]))) < 4e-3
