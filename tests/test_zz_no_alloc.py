"""mps_heev_noalloc (the eigen-solver on caller-owned device buffers, every
intermediate in the library's static device array) against mps_heev on the
same matrices: two calls in a row, the second smaller, so the second reuses
the array the first left behind.  Both run the same kernels on the same
input: eigenvalues and eigenvectors must agree bit for bit, and both must
diagonalise A to the eigen-solver tests' bar (residual and orthogonality
within 16 n u)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2502_19289_amd")


def _hip():
    """The HIP runtime libctebd.so itself links (not the one PyTorch ships):
    symbol lookup through the library's handle searches its dependencies."""
    P.load()  # starts the runtimes in the order the binding needs
    h = C.CDLL(P.ffi.LIB_PATH)
    h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    h.hipFree.argtypes = [C.c_void_p]
    h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    h.hipDeviceSynchronize.argtypes = []
    return h


H2D, D2H = 1, 2


def _hermitian(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    # graded spectrum, as the Gram matrices of the splits have
    Q, _ = np.linalg.qr(X)
    lam = np.exp(-np.linspace(0, 30, n)) * rng.uniform(0.5, 1.5, n)
    return (Q * lam) @ Q.conj().T


def test_noalloc_heev_matches_heev():
    hip = _hip()
    lib = P.load()
    for n in (512, 181):  # the largest size first, then a smaller one into the used array
        A = np.ascontiguousarray(_hermitian(n, seed=n))
        A = (A + A.conj().T) / 2
        w_ref, V_ref = P.heev(A)
        ptrs = []
        for nbytes in (A.nbytes, 8 * n, 16 * n * n):
            p = C.c_void_p()
            assert hip.hipMalloc(C.byref(p), nbytes) == 0
            ptrs.append(p)
        dA, dw, dV = ptrs
        try:
            assert hip.hipMemcpy(dA, A.ctypes.data, A.nbytes, H2D) == 0
            st = lib.mps_heev_noalloc(n, dA, dw, dV, None)
            assert st == 0, lib.mps_last_error(None).decode()
            w = np.zeros(n)
            V = np.zeros((n, n), dtype=np.complex128)
            assert hip.hipMemcpy(w.ctypes.data, dw, w.nbytes, D2H) == 0
            assert hip.hipMemcpy(V.ctypes.data, dV, V.nbytes, D2H) == 0
        finally:
            for p in ptrs:
                hip.hipFree(p)
        assert np.array_equal(w, w_ref)
        assert np.array_equal(V, V_ref)
        u = 2.0 ** -53
        nrm = np.abs(w).max()
        assert np.abs(A @ V - V * w).max() <= 16 * n * u * nrm
        assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 16 * n * u
        assert np.all(np.diff(w) >= 0)


def test_noalloc_heev_rejects_sizes_beyond_its_array():
    lib = P.load()
    assert lib.mps_heev_noalloc(513, C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), None) == -1
    assert "512" in lib.mps_last_error(None).decode()
    assert lib.mps_heev_noalloc(0, C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), None) == -1
