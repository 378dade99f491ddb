"""MI355X-native (gfx950) adjoint Monte Carlo for optimal control of jump-diffusions.

The hot path (forward Euler-Maruyama sweep, discrete adjoint sweep, FP64 Monte
Carlo reductions, Armijo gradient iteration) runs in hand-written HIP kernels
behind the C-ABI library ``libjd.so`` (declared in ``include/jd.h``).  The
Python modules here only marshal arguments: ``binding`` (ctypes), ``autograd``
(torch.autograd.Function), ``serving`` (request loop) and ``workloads``
(seeded synthetic inputs).
"""

__all__ = ["binding", "workloads"]
