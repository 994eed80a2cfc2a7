"""ctypes binding of libctebd.so (argument marshalling only).

Every function of include/cluster_tebd.h is exposed with the same name; the
``MPS`` class wraps a handle.  The library is loaded from this package's
directory; importing fails loudly when it has not been built (there is no
fallback implementation).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctebd.so")

MPS_OK, MPS_EINVAL, MPS_ENOMEM, MPS_ESPAN, MPS_ENOTUNITARY, MPS_EDEVICE, MPS_ESTATE, MPS_EIO = \
    0, -1, -2, -3, -4, -5, -6, -7
PREC = {"fp64": 0, "fp32": 1, "bf16x6": 2}
SVD = {"exact": 0, "learned": 1}
BATCH = {"none": 0, "step": 1, "wave": 2}
EIG = {"auto": 0, "jacobi": 1, "tridiag": 2}


class Options(C.Structure):
    _fields_ = [("k_max", C.c_int), ("q_max", C.c_int), ("l_max", C.c_int),
                ("precision", C.c_int), ("svd_mode", C.c_int), ("batch", C.c_int),
                ("eig_method", C.c_int), ("floor_c", C.c_double), ("hip_stream", C.c_void_p)]


class GateC(C.Structure):
    _fields_ = [("nq", C.c_int), ("q", C.c_int * 2), ("u", C.c_double * 32)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("cluster_updates", C.c_int64), ("svds", C.c_int64),
                ("site_updates", C.c_int64), ("sketch_accepted", C.c_int64),
                ("sketch_fallback", C.c_int64), ("jacobi_sweeps", C.c_int64),
                ("discarded_weight", C.c_double)]


class CtebdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


EXPORTS = ["mps_default_options", "mps_create", "mps_destroy", "mps_apply_cluster", "mps_set_options", "mps_dmrg_step",
           "mps_save", "mps_load",
           "mps_run_layer", "mps_flush", "mps_queue_layer", "mps_step", "mps_run_steps", "mps_clone", "mps_overlap",
           "mps_fidelity", "mps_bond_dims", "mps_schmidt",
           "mps_export_site", "mps_import", "mps_amplitudes", "mps_get_stats",
           "mps_set_timing", "mps_set_burst_timing", "mps_kernel_dispatches", "mps_kernel_times", "mps_kernel_bytes", "mps_heev", "mps_heev_noalloc", "mps_last_error", "mps_plan",
           "mlp_num_params", "mlp_create", "mlp_destroy", "mlp_get_params", "mlp_set_params",
           "mlp_forward", "mlp_grad", "mlp_train", "mps_set_sketch_model", "mps_svd_log", "mps_sketch_range"]
N_FEAT = 12

_lib = None


def _start_torch_hip() -> None:
    """PyTorch's ROCm wheel carries its own HIP runtime.  Once this library's
    runtime has started in a process, torch no longer finds a GPU there, so
    where torch is installed its runtime is started first (the other order
    works)."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load(path: str = LIB_PATH) -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2502_19289_amd.build`")
    _start_torch_hip()
    lib = C.CDLL(path)
    P, I, D = C.c_void_p, C.c_int, C.c_double
    lib.mps_default_options.argtypes = [C.POINTER(Options)]
    lib.mps_create.argtypes = [I, I, D, C.POINTER(Options), C.POINTER(P)]
    lib.mps_destroy.argtypes = [P]
    lib.mps_apply_cluster.argtypes = [P, C.POINTER(I), I, C.POINTER(D)]
    lib.mps_run_layer.argtypes = [P, C.POINTER(GateC), I]
    lib.mps_flush.argtypes = [P]
    lib.mps_queue_layer.argtypes = [P, C.POINTER(GateC), I]
    lib.mps_step.argtypes = [P, C.POINTER(I), C.POINTER(I)]
    lib.mps_run_steps.argtypes = [P, I, C.POINTER(I), C.POINTER(I)]
    lib.mps_clone.argtypes = [P, C.POINTER(Options), C.POINTER(P)]
    lib.mps_set_options.argtypes = [P, C.POINTER(Options)]
    lib.mps_dmrg_step.argtypes = [P, C.POINTER(GateC), C.POINTER(I), I, I, I, I, C.POINTER(D)]
    lib.mps_save.argtypes = [P, C.c_char_p]
    lib.mps_load.argtypes = [C.c_char_p, C.POINTER(P)]
    lib.mps_overlap.argtypes = [P, P, C.POINTER(D), C.POINTER(D)]
    lib.mps_fidelity.argtypes = [P, C.POINTER(D), C.POINTER(D)]
    lib.mps_bond_dims.argtypes = [P, C.POINTER(I)]
    lib.mps_schmidt.argtypes = [P, I, C.POINTER(D), I, C.POINTER(I)]
    lib.mps_export_site.argtypes = [P, I, C.POINTER(D), C.c_int64, C.POINTER(I)]
    lib.mps_import.argtypes = [P, C.POINTER(I), C.POINTER(C.POINTER(D)), C.POINTER(C.POINTER(D)), D]
    lib.mps_amplitudes.argtypes = [P, C.POINTER(D), C.c_int64]
    lib.mps_get_stats.argtypes = [P, C.POINTER(Stats)]
    lib.mps_set_timing.argtypes = [P, I]
    lib.mps_kernel_times.argtypes = [P, C.POINTER(D), C.POINTER(C.c_int64), C.POINTER(D), I, C.c_char_p, I,
                                     C.POINTER(I)]
    lib.mps_kernel_bytes.argtypes = [P, C.POINTER(D), I, C.POINTER(I)]
    lib.mps_set_burst_timing.argtypes = [P, C.c_char_p, I, I]
    lib.mps_kernel_dispatches.argtypes = [P, C.POINTER(C.c_int64), I, C.POINTER(I)]
    lib.mps_heev.argtypes = [I, C.POINTER(D), C.POINTER(D), C.POINTER(D)]
    lib.mps_heev_noalloc.argtypes = [I, P, P, P, P]
    lib.mps_last_error.argtypes = [P]
    lib.mps_last_error.restype = C.c_char_p
    lib.mps_plan.argtypes = [I, I, I, I, C.POINTER(I), C.POINTER(GateC), C.POINTER(I), I, I,
                             C.POINTER(I), C.POINTER(I), I, C.POINTER(I), C.POINTER(I)]
    F = C.POINTER(C.c_float)
    lib.mlp_num_params.argtypes = []
    lib.mlp_create.argtypes = [I, C.POINTER(P)]
    lib.mlp_destroy.argtypes = [P]
    lib.mlp_get_params.argtypes = [P, F]
    lib.mlp_set_params.argtypes = [P, F]
    lib.mlp_forward.argtypes = [P, F, I, F]
    lib.mlp_grad.argtypes = [P, F, F, I, C.c_float, F, F]
    lib.mlp_train.argtypes = [P, F, F, I, I, I, C.c_float, C.c_float, C.c_uint64, F]
    lib.mps_set_sketch_model.argtypes = [P, P]
    lib.mps_svd_log.argtypes = [P, F, F, I, C.POINTER(I)]
    lib.mps_sketch_range.argtypes = [P, I, I, C.POINTER(D), C.POINTER(D), C.POINTER(D), C.POINTER(D), C.POINTER(D),
                                     C.POINTER(D), C.POINTER(I)]
    for name in EXPORTS:
        if name != "mps_last_error":
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def make_gates(gates: Iterable[Tuple[Sequence[int], np.ndarray]]):
    """[(qubits, matrix)] -> ctypes array of GateC."""
    gl = list(gates)
    arr = (GateC * max(1, len(gl)))()
    for i, (q, u) in enumerate(gl):
        u = np.asarray(u, dtype=np.complex128)
        arr[i].nq = len(q)
        for j, qq in enumerate(q):
            arr[i].q[j] = int(qq)
        flat = np.zeros(32)
        v = u.reshape(-1)
        flat[0:2 * v.size:2] = v.real
        flat[1:2 * v.size:2] = v.imag
        arr[i].u[:] = flat.tolist()
    return arr, len(gl)


def default_options() -> Options:
    o = Options()
    load().mps_default_options(C.byref(o))
    return o


class MPS:
    """An n-qubit MPS living on the GPU (handle of libctebd.so)."""

    def __init__(self, n: int, chi_max: int, eps: float, k_max: int = 4, precision: str = "fp32",
                 batch: str = "step", svd: str = "exact", q_max: int = 0, l_max: int = 0,
                 floor_c: float = 4.0, hip_stream: Optional[int] = None, eig: str = "auto"):
        self.lib = load()
        o = default_options()
        o.k_max, o.q_max, o.l_max = k_max, q_max, l_max
        o.precision, o.batch, o.svd_mode = PREC[precision], BATCH[batch], SVD[svd]
        o.eig_method = EIG[eig]
        o.floor_c = floor_c
        o.hip_stream = hip_stream
        h = C.c_void_p()
        st = self.lib.mps_create(n, chi_max, eps, C.byref(o), C.byref(h))
        if st != MPS_OK:
            raise CtebdError(st, self.lib.mps_last_error(None).decode())
        self._opt = o
        self.h = h
        self.n = n

    def _check(self, st: int):
        if st != MPS_OK:
            raise CtebdError(st, self.lib.mps_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.mps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_cluster(self, qubits: Sequence[int], U: np.ndarray):
        q = np.ascontiguousarray(qubits, dtype=np.int32)
        u = np.ascontiguousarray(np.asarray(U, dtype=np.complex128)).view(np.float64)
        self._check(self.lib.mps_apply_cluster(self.h, _iptr(q), len(q), _dptr(u)))

    def run_layer(self, gates: Iterable[Tuple[Sequence[int], np.ndarray]]):
        arr, ng = make_gates(gates)
        self._check(self.lib.mps_run_layer(self.h, arr, ng))

    def flush(self):
        self._check(self.lib.mps_flush(self.h))

    def queue_layer(self, gates: Iterable[Tuple[Sequence[int], np.ndarray]]):
        arr, ng = make_gates(gates)
        self._check(self.lib.mps_queue_layer(self.h, arr, ng))

    def step(self) -> Tuple[int, int]:
        """Executes one cluster-TEBD step; returns (clusters, sub-layers left)."""
        c, r = C.c_int(), C.c_int()
        self._check(self.lib.mps_step(self.h, C.byref(c), C.byref(r)))
        return c.value, r.value

    def run_steps(self, nsteps: int) -> Tuple[int, int]:
        """mps_run_steps: the next nsteps steps; returns (clusters, sub-layers left)."""
        c, r = C.c_int(), C.c_int()
        self._check(self.lib.mps_run_steps(self.h, int(nsteps), C.byref(c), C.byref(r)))
        return c.value, r.value

    def clone(self, precision: Optional[str] = None, batch: Optional[str] = None,
              eig: Optional[str] = None) -> "MPS":
        o = Options()
        o.k_max, o.q_max, o.l_max = self._opt.k_max, self._opt.q_max, self._opt.l_max
        o.precision = PREC[precision] if precision else self._opt.precision
        o.batch = BATCH[batch] if batch else self._opt.batch
        o.eig_method = EIG[eig] if eig else self._opt.eig_method
        o.svd_mode, o.floor_c, o.hip_stream = self._opt.svd_mode, self._opt.floor_c, None
        h = C.c_void_p()
        self._check(self.lib.mps_clone(self.h, C.byref(o), C.byref(h)))
        m = MPS.__new__(MPS)
        m.lib, m.h, m.n, m._opt = self.lib, h, self.n, o
        return m

    def options(self) -> dict:
        o = self._opt
        inv = lambda d, v: next(k for k, x in d.items() if x == v)  # noqa: E731
        return {"k_max": o.k_max, "q_max": o.q_max, "l_max": o.l_max, "precision": inv(PREC, o.precision),
                "batch": inv(BATCH, o.batch), "svd": inv(SVD, o.svd_mode), "eig": inv(EIG, o.eig_method),
                "floor_c": o.floor_c}

    def set_options(self, k_max: Optional[int] = None, q_max: Optional[int] = None, l_max: Optional[int] = None,
                    precision: Optional[str] = None, batch: Optional[str] = None, svd: Optional[str] = None,
                    eig: Optional[str] = None, floor_c: Optional[float] = None, hip_stream: Optional[int] = None):
        """mps_set_options: fields left at None keep their current value."""
        o = Options()
        C.memmove(C.byref(o), C.byref(self._opt), C.sizeof(Options))
        if k_max is not None:
            o.k_max = k_max
        if q_max is not None:
            o.q_max = q_max
        if l_max is not None:
            o.l_max = l_max
        if precision is not None:
            o.precision = PREC[precision]
        if batch is not None:
            o.batch = BATCH[batch]
        if svd is not None:
            o.svd_mode = SVD[svd]
        if eig is not None:
            o.eig_method = EIG[eig]
        if floor_c is not None:
            o.floor_c = floor_c
        o.hip_stream = hip_stream
        self._check(self.lib.mps_set_options(self.h, C.byref(o)))
        self._opt = o

    def dmrg_step(self, layers, chi_max_dmrg: int, q_max: int, sweeps: int = 2) -> float:
        """mps_dmrg_step: one adaptive-grouping DMRG step over `layers` (lists of
        (qubits, matrix)); returns the fit's fidelity."""
        flat = [g for layer in layers for g in layer]
        arr, _ = make_gates(flat)
        ll = np.array([len(layer) for layer in layers], dtype=np.int32)
        f = C.c_double()
        self._check(self.lib.mps_dmrg_step(self.h, arr, _iptr(ll), len(layers), int(chi_max_dmrg), int(q_max),
                                           int(sweeps), C.byref(f)))
        return f.value

    def save(self, path: str):
        """mps_save: the whole handle to a file."""
        self._check(self.lib.mps_save(self.h, os.fsencode(path)))

    @classmethod
    def load(cls, path: str) -> "MPS":
        """mps_load: a new handle from a file written by save()."""
        lib = load()
        h = C.c_void_p()
        st = lib.mps_load(os.fsencode(path), C.byref(h))
        if st != MPS_OK:
            raise CtebdError(st, lib.mps_last_error(None).decode())
        m = MPS.__new__(MPS)
        m.lib, m.h = lib, h
        # the saved n and options, read back from the file's header
        with open(path, "rb") as f:
            head = f.read(8 + 4 + 4 + 4 + 8 + 7 * 4 + 8)
        n = int.from_bytes(head[12:16], "little", signed=True)
        vals = np.frombuffer(head[28:56], dtype="<i4")
        o = Options()
        o.k_max, o.q_max, o.l_max, o.precision, o.svd_mode, o.batch, o.eig_method = (int(v) for v in vals)
        o.floor_c = float(np.frombuffer(head[56:64], dtype="<f8")[0])
        o.hip_stream = None
        m.n, m._opt = n, o
        return m

    def overlap(self, other: "MPS") -> complex:
        re, im = C.c_double(), C.c_double()
        self._check(self.lib.mps_overlap(self.h, other.h, C.byref(re), C.byref(im)))
        return complex(re.value, im.value)

    def infidelity(self, other: "MPS") -> float:
        """1 - |<a|b>|^2 / (<a|a><b|b>), computed on the device in FP64."""
        ab = abs(self.overlap(other)) ** 2
        return 1.0 - ab / (self.overlap(self).real * other.overlap(other).real)

    def fidelity(self) -> Tuple[float, float]:
        f, lf = C.c_double(), C.c_double()
        self._check(self.lib.mps_fidelity(self.h, C.byref(f), C.byref(lf)))
        return f.value, lf.value

    def bond_dims(self) -> List[int]:
        a = np.zeros(self.n - 1, dtype=np.int32)
        self._check(self.lib.mps_bond_dims(self.h, _iptr(a)))
        return a.tolist()

    def schmidt(self, bond: int) -> np.ndarray:
        ln = C.c_int()
        self._check(self.lib.mps_schmidt(self.h, bond, None, 0, C.byref(ln)))
        a = np.zeros(max(1, ln.value))
        self._check(self.lib.mps_schmidt(self.h, bond, _dptr(a), a.size, C.byref(ln)))
        return a[: ln.value]

    def site(self, j: int) -> np.ndarray:
        dims = np.zeros(3, dtype=np.int32)
        self._check(self.lib.mps_export_site(self.h, j, None, 0, _iptr(dims)))
        cnt = int(dims[0]) * 2 * int(dims[2])
        buf = np.zeros(2 * cnt)
        self._check(self.lib.mps_export_site(self.h, j, _dptr(buf), cnt, _iptr(dims)))
        return buf.view(np.complex128).reshape(int(dims[0]), 2, int(dims[2]))

    def sites(self) -> List[np.ndarray]:
        return [self.site(j) for j in range(self.n)]

    def import_state(self, B: Sequence[np.ndarray], lam: Sequence[np.ndarray], log_f: float = 0.0):
        chi = np.array([b.shape[2] for b in B[:-1]], dtype=np.int32)
        sb = [np.ascontiguousarray(np.asarray(b, dtype=np.complex128)).view(np.float64) for b in B]
        lb = [np.ascontiguousarray(np.asarray(l, dtype=np.float64)) for l in lam]
        sp = (C.POINTER(C.c_double) * len(sb))(*[_dptr(x) for x in sb])
        lp = (C.POINTER(C.c_double) * len(lb))(*[_dptr(x) for x in lb])
        self._check(self.lib.mps_import(self.h, _iptr(chi), sp, lp, log_f))

    def amplitudes(self) -> np.ndarray:
        buf = np.zeros(2 << self.n)
        self._check(self.lib.mps_amplitudes(self.h, _dptr(buf), 1 << self.n))
        return buf.view(np.complex128)

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.mps_get_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def set_timing(self, on: bool = True):
        self._check(self.lib.mps_set_timing(self.h, int(on)))

    def set_burst_timing(self, kernel_class: Optional[str], stride: int = 1, reps: int = 0):
        """Time `kernel_class` by bursts of reps + 1 launches on every stride-th
        launch (None: off); see mps_set_burst_timing."""
        name = kernel_class.encode() if kernel_class else None
        self._check(self.lib.mps_set_burst_timing(self.h, name, int(stride), int(reps)))

    def kernel_dispatches(self) -> dict:
        """{class: kernel dispatches since timing was switched on, burst re-launches included}."""
        cnt = C.c_int()
        d = np.zeros(64, dtype=np.int64)
        self._check(self.lib.mps_kernel_dispatches(self.h, d.ctypes.data_as(C.POINTER(C.c_int64)), 64,
                                                   C.byref(cnt)))
        names = C.create_string_buffer(4096)
        self._check(self.lib.mps_kernel_times(self.h, None, None, None, 0, names, 4096, C.byref(cnt)))
        nm = names.value.decode().split(",") if cnt.value else []
        return {n: int(d[i]) for i, n in enumerate(nm)}

    def kernel_times(self) -> dict:
        """{class: (ms, launches, algorithmic flops, algorithmic HBM bytes)} since
        timing was switched on."""
        cnt = C.c_int()
        ms = np.zeros(64)
        fl = np.zeros(64)
        by = np.zeros(64)
        la = np.zeros(64, dtype=np.int64)
        names = C.create_string_buffer(4096)
        self._check(self.lib.mps_kernel_times(self.h, _dptr(ms), la.ctypes.data_as(C.POINTER(C.c_int64)),
                                              _dptr(fl), 64, names, 4096, C.byref(cnt)))
        self._check(self.lib.mps_kernel_bytes(self.h, _dptr(by), 64, C.byref(cnt)))
        nm = names.value.decode().split(",") if cnt.value else []
        return {n: (float(ms[i]), int(la[i]), float(fl[i]), float(by[i])) for i, n in enumerate(nm)}


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class KeptRankNet:
    """The kept-rank network of the learned sketch (device-resident, FP32)."""

    def __init__(self, seed: int = 0):
        self.lib = load()
        h = C.c_void_p()
        st = self.lib.mlp_create(seed, C.byref(h))
        if st != MPS_OK:
            raise CtebdError(st, "mlp_create failed")
        self.h = h
        self.n_params = self.lib.mlp_num_params()

    def _check(self, st):
        if st != MPS_OK:
            raise CtebdError(st, "network call failed")

    def close(self):
        if getattr(self, "h", None):
            self.lib.mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        p = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.lib.mlp_get_params(self.h, _fptr(p)))
        return p

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._check(self.lib.mlp_set_params(self.h, _fptr(p)))

    def forward(self, X: np.ndarray) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.zeros(X.shape[0], dtype=np.float32)
        self._check(self.lib.mlp_forward(self.h, _fptr(X), X.shape[0], _fptr(y)))
        return y

    def grad(self, X: np.ndarray, t: np.ndarray, tau: float):
        X = np.ascontiguousarray(X, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_float()
        self._check(self.lib.mlp_grad(self.h, _fptr(X), _fptr(t), X.shape[0], tau, _fptr(g), C.byref(loss)))
        return g, loss.value

    def train(self, X, t, epochs=50, batch=256, lr=3e-3, tau=0.9, seed=0) -> float:
        X = np.ascontiguousarray(X, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        loss = C.c_float()
        self._check(self.lib.mlp_train(self.h, _fptr(X), _fptr(t), X.shape[0], epochs, batch, lr, tau, seed,
                                       C.byref(loss)))
        return loss.value


def attach_model(mps: "MPS", net: Optional[KeptRankNet]):
    st = load().mps_set_sketch_model(mps.h, net.h if net is not None else None)
    if st != MPS_OK:
        raise CtebdError(st, "mps_set_sketch_model failed")


def svd_log(mps: "MPS"):
    """Moves the (features, log2 kept rank) pairs logged by `mps` out of it."""
    lib = load()
    cnt = C.c_int()
    lib.mps_svd_log(mps.h, None, None, 0, C.byref(cnt))
    n = cnt.value
    X = np.zeros((max(n, 1), N_FEAT), dtype=np.float32)
    t = np.zeros(max(n, 1), dtype=np.float32)
    lib.mps_svd_log(mps.h, _fptr(X), _fptr(t), n, C.byref(cnt))
    return X[:n], t[:n]


def sketch_range(mps: "MPS", G: np.ndarray, omega: np.ndarray, probes: np.ndarray):
    """mps_sketch_range: the device range finder on G with the given test and
    probe matrices; returns (mu, V, est, trace, accepted)."""
    lib = load()
    G = np.ascontiguousarray(G, dtype=np.complex128)
    omega = np.ascontiguousarray(omega, dtype=np.complex128)
    probes = np.ascontiguousarray(probes, dtype=np.complex128)
    n, s = omega.shape
    mu = np.zeros(s)
    V = np.zeros((n, s), dtype=np.complex128)
    est = np.zeros(2)
    acc = C.c_int()
    st = lib.mps_sketch_range(mps.h, n, s, _dptr(G.view(np.float64)), _dptr(omega.view(np.float64)),
                              _dptr(probes.view(np.float64)), _dptr(mu), _dptr(V.view(np.float64)), _dptr(est),
                              C.byref(acc))
    if st != MPS_OK:
        raise CtebdError(st, lib.mps_last_error(mps.h).decode())
    return mu, V, float(est[0]), float(est[1]), bool(acc.value)


def plan(n: int, k_max: int, layers, chi: Sequence[int], start: int = 0, q_max: int = 0, l_max: int = 0):
    """Host planner (mps_plan): returns (end, clusters, n_sub)."""
    lib = load()
    flat = [g for l in layers for g in l]
    arr, ng = make_gates(flat)
    ll = np.array([len(l) for l in layers], dtype=np.int32)
    ch = np.ascontiguousarray(chi, dtype=np.int32)
    end, cnt, nsub = C.c_int(), C.c_int(), C.c_int()
    out = np.zeros(2 * n, dtype=np.int32)
    st = lib.mps_plan(n, k_max, q_max, l_max, _iptr(ch), arr, _iptr(ll), len(layers), start,
                      C.byref(end), _iptr(out), n, C.byref(cnt), C.byref(nsub))
    if st != MPS_OK:
        raise CtebdError(st, lib.mps_last_error(None).decode())
    cl = [(int(out[2 * i]), int(out[2 * i + 1])) for i in range(cnt.value)]
    return end.value, cl, nsub.value


def heev(A: np.ndarray):
    """Eigen-decomposition of a Hermitian matrix on the GPU by the tridiagonal
    divide-and-conquer solver of the large splits: (w ascending, V columns)."""
    lib = load()
    a = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("square matrix expected")
    w = np.zeros(n)
    V = np.zeros((n, n), dtype=np.complex128)
    st = lib.mps_heev(n, _dptr(a.view(np.float64)), _dptr(w), _dptr(V.view(np.float64)))
    if st != MPS_OK:
        raise CtebdError(st, lib.mps_last_error(None).decode())
    return w, V
