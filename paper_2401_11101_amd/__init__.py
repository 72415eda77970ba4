"""MI355X laminography: Fourier-route FBP, forward projector L and adjoint L*.

The operators run in the HIP library `lib/liblamino.so` (C ABI in
include/lamino.h); this package marshals torch tensors into it.
"""
from ._abi import LaminoError, load_library  # noqa: F401


def __getattr__(name):
    # lazy imports so that `import paper_2401_11101_amd` never touches torch.cuda
    if name == "Plan":
        from .plan import Plan

        return Plan
    if name in ("LaminoL", "LaminoLstar", "cgls"):
        from . import autograd

        return getattr(autograd, name)
    if name in ("admm_tv", "AdmmTV"):
        from . import tv

        return getattr(tv, name)
    if name == "Server":
        from .serve import Server

        return Server
    raise AttributeError(name)
