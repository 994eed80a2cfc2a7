"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function the header declares, and its planner (host C++) agrees with
the oracle's independent planner step by step."""
import os
import re

import numpy as np
import pytest

from oracle import planner as PL
from workloads import random_structured

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2502_19289_amd import ffi
    return ffi


def test_exports_every_declared_symbol():
    ffi = _lib()
    lib = ffi.load()
    header = open(os.path.join(ROOT, "include", "cluster_tebd.h")).read()
    declared = set(re.findall(r"^\s*(?:const char\*|mps_status|int)\s+((?:mps|mlp)_\w+)\s*\(", header, re.M))
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(ffi.EXPORTS)


def test_create_without_gpu_fails_cleanly():
    ffi = _lib()
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(ffi.CtebdError) as e:
        ffi.MPS(8, 4, 1e-12)
    assert e.value.status == ffi.MPS_EDEVICE
    assert "no HIP device" in str(e.value)  # through mps_last_error(NULL)


@pytest.mark.parametrize("n,chi,eps", [(1, 4, 1e-12), (8, 0, 1e-12), (8, 4096, 1e-12), (8, 4, -1.0),
                                       (8, 4, float("nan"))])
def test_create_rejects_bad_sizes_with_a_message(n, chi, eps):
    ffi = _lib()
    with pytest.raises(ffi.CtebdError) as e:
        ffi.MPS(n, chi, eps)
    assert e.value.status == ffi.MPS_EINVAL
    assert "chi_max <= 2048" in str(e.value)


def _layers_for_abi(c):
    from paper_2502_19289_amd.gates import GATES
    return [[(g.qubits, GATES[g.name]) for g in l] for l in c.layers]


@pytest.mark.parametrize("seed,k_max,q_max,l_max", [(0, 2, 0, 0), (1, 3, 0, 0), (2, 5, 0, 0),
                                                    (3, 4, 9, 0), (4, 6, 12, 3), (5, 8, 0, 2)])
def test_planner_matches_oracle(seed, k_max, q_max, l_max):
    ffi = _lib()
    n = 48
    c = random_structured(n, 12, 10, ("H", "S", "CNOT"), 0.15, seed=seed, workload_id=31)
    layers = _layers_for_abi(c)
    subs = PL.legalize(c.layers, k_max)
    rng = np.random.default_rng(seed)
    start, steps = 0, 0
    while start < len(subs):
        chi = [int(min(2 ** rng.integers(0, 5), 2 ** min(b + 1, n - b - 1))) for b in range(n - 1)]
        qm = q_max if q_max > 0 else 62
        lm = l_max if l_max > 0 else 1 << 30
        e_o, cl_o = PL.plan_step(subs, start, n, chi, k_max, qm, lm)
        e_c, cl_c, nsub = ffi.plan(n, k_max, layers, chi, start=start, q_max=q_max, l_max=l_max)
        assert nsub == len(subs)
        assert e_c == e_o
        assert cl_c == [tuple(x) for x in cl_o]
        start = e_o
        steps += 1
    assert steps > 3


def test_load_rejects_missing_and_corrupt_files(tmp_path):
    """mps_load reads and checks the whole file on the host before it creates
    a handle, so these errors need no GPU."""
    ffi = _lib()
    with pytest.raises(ffi.CtebdError) as e:
        ffi.MPS.load(str(tmp_path / "absent.ctebd"))
    assert e.value.status == ffi.MPS_EIO
    junk = tmp_path / "junk.ctebd"
    junk.write_bytes(b"not a saved state at all, just some bytes" * 3)
    with pytest.raises(ffi.CtebdError) as e:
        ffi.MPS.load(str(junk))
    assert e.value.status == ffi.MPS_EIO
    # the right magic with a wrong checksum
    bad = tmp_path / "bad.ctebd"
    bad.write_bytes(b"CTEBDMPS" + bytes(64))
    with pytest.raises(ffi.CtebdError) as e:
        ffi.MPS.load(str(bad))
    assert e.value.status == ffi.MPS_EIO
    assert "checksum" in str(e.value)
