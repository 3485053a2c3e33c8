"""MI355X (gfx950) implementation of one pressure-based time step of the
discrete-forcing immersed boundary method for compressible flow with heat
exchange (Riahi, Goncalves da Silva, Meldi).

The numerical work runs in the HIP library ``libibm_hip.so`` behind the C ABI of
``include/ibm.h``; ``solver.IBMSolver`` marshals torch device tensors into it.
Importing this package does not load the library; ``IBMSolver`` does, and fails
loudly when it has not been built.
"""

__all__ = ["inputs", "IBMSolver"]


def __getattr__(name):
    if name == "IBMSolver":
        from .solver import IBMSolver
        return IBMSolver
    raise AttributeError(name)
