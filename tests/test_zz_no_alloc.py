"""The allocation-free statistics-and-samples entry point against the
ordinary one (sv_moments_sample), through the C ABI: the same kernels, so
samples and statistics must agree bit for bit, on two calls in a row (the
second on a smaller input, over the scratch the first left behind)."""
import ctypes

import numpy as np
import pytest

from paper_1608_00263_amd import circuits as C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1608_00263_amd import sv  # noqa: E402


def _both(st, k, seed):
    L = sv.lib()
    ref = sv.Stats()
    ref_x = torch.zeros(max(k, 1), dtype=torch.int64, device="cuda")
    sv.check(L.sv_moments_sample(st.h, ctypes.byref(ref), k, ctypes.c_uint64(seed),
                                 ctypes.c_void_p(ref_x.data_ptr()), 1))
    got = sv.Stats()
    got_x = torch.full((max(k, 1),), -1, dtype=torch.int64, device="cuda")
    sv.check(L.sv_moments_sample_noalloc(st.h, ctypes.byref(got), k, ctypes.c_uint64(seed),
                                         ctypes.c_void_p(got_x.data_ptr()) if k else None))
    return ref.as_dict(), ref_x[:k].cpu().numpy(), got.as_dict(), got_x[:k].cpu().numpy()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_matches_moments_sample_twice(dtype):
    npdt = np.complex64 if dtype == "c64" else np.complex128
    # first call: 22 qubits, 2e5 samples, some zero amplitudes
    psi = C.random_state(22, 110, dtype=npdt)
    psi[np.random.default_rng(3).choice(psi.size, 100, replace=False)] = 0
    st = sv.State(22, dtype, tensor=torch.from_numpy(psi).to("cuda"))
    ref, rx, got, gx = _both(st, 200000, 77)
    np.testing.assert_array_equal(gx, rx)
    for key in ("norm", "entropy", "unif_ce", "zero_count"):
        assert got[key] == ref[key], key
    np.testing.assert_array_equal(got["moments"], ref["moments"])
    assert got["zero_count"] == 100
    st.close()
    # second call: a smaller state and fewer samples over the same scratch
    psi2 = C.random_state(15, 111, dtype=npdt)
    st2 = sv.State(15, dtype, tensor=torch.from_numpy(psi2).to("cuda"))
    ref, rx, got, gx = _both(st2, 3000, 78)
    np.testing.assert_array_equal(gx, rx)
    for key in ("norm", "entropy", "unif_ce", "zero_count"):
        assert got[key] == ref[key], key
    np.testing.assert_array_equal(got["moments"], ref["moments"])
    # statistics only
    ref0, _, got0, _ = _both(st2, 0, 1)
    assert got0["entropy"] == ref0["entropy"]
    st2.close()


def test_noalloc_limits():
    L = sv.lib()
    st = sv.State(20, "c64")
    st.reset()
    s = sv.Stats()
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    # 10^7 samples need 120 MB of scratch: refused before any device work
    assert L.sv_moments_sample_noalloc(st.h, ctypes.byref(s), 10 ** 7, ctypes.c_uint64(1),
                                       ctypes.c_void_p(out.data_ptr())) == sv.SV_ERANGE
    assert L.sv_moments_sample_noalloc(st.h, None, 4, ctypes.c_uint64(1),
                                       ctypes.c_void_p(out.data_ptr())) == sv.SV_EINVAL
    assert L.sv_moments_sample_noalloc(st.h, ctypes.byref(s), 4, ctypes.c_uint64(1), None) == sv.SV_EINVAL
    assert L.sv_moments_sample_noalloc(st.h, ctypes.byref(s), -1, ctypes.c_uint64(1), None) == sv.SV_ERANGE
    st.close()
