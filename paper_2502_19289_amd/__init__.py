"""MI355X cluster-TEBD (arXiv:2502.19289): Python front end of libctebd.so.

The hot path (cluster unitaries, merges, truncated-SVD splits, fidelity
bookkeeping) runs in the HIP kernels of the library; this package only
marshals arguments.  Importing it requires the built library.
"""
from .ffi import MPS, CtebdError, heev, load, plan  # noqa: F401
from .gates import GATES  # noqa: F401


def run_circuit(mps: "MPS", layers, flush: bool = True) -> None:
    """Feeds circuit layers (lists of objects with ``name`` and ``qubits``) to
    ``mps`` one layer at a time; the library decides the steps."""
    for layer in layers:
        mps.run_layer([(g.qubits, GATES[g.name]) for g in layer])
    if flush:
        mps.flush()
