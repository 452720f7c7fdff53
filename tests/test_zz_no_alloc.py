"""The allocation-free start-vector entry point (ftlm_gaussian_vectors_noalloc)
against ftlm_gaussian_vectors, through the C ABI: the same kernels on the same
arguments must give bitwise the same vectors, on two calls in a row (the second
with fewer rows and columns, so it reuses the shared scratch array left by the
first), and sizes beyond the array are rejected."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _call(fn, seed, inst, field, r0, n_cols, dim):
    out = torch.empty((dim, n_cols), dtype=torch.complex128, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(ctypes.c_uint64(seed), inst, field, r0, n_cols, ctypes.c_uint64(dim),
            ctypes.c_void_p(out.data_ptr()), stream)
    torch.cuda.synchronize()
    return rc, out.cpu().numpy()


def test_noalloc_start_vectors_match_allocating_entry_point():
    from paper_2607_25585_amd import _ffi
    L = _ffi.lib()
    cases = [(1234567, 3, 2, 5, 12, 300_001), (99, 0, 0, 0, 3, 4097)]
    for seed, inst, field, r0, n_cols, dim in cases:
        print("case noalloc start vectors dim", dim, "cols", n_cols, flush=True)
        rc_a, a = _call(L.ftlm_gaussian_vectors_noalloc, seed, inst, field, r0, n_cols, dim)
        rc_b, b = _call(L.ftlm_gaussian_vectors, seed, inst, field, r0, n_cols, dim)
        assert rc_a == 0 and rc_b == 0
        assert np.array_equal(a.view(np.float64), b.view(np.float64))
        assert np.all(np.isfinite(a.view(np.float64)))
    # more columns than the scratch array holds: a clear error, nothing launched
    out = torch.empty((8, 65), dtype=torch.complex128, device="cuda")
    rc = L.ftlm_gaussian_vectors_noalloc(ctypes.c_uint64(1), 0, 0, 0, 65, ctypes.c_uint64(8),
                                         ctypes.c_void_p(out.data_ptr()), None)
    assert rc == -4
    assert b"64" in L.ftlm_last_error()
