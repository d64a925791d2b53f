"""MI355X-native hot path of the Open Earth Compiler's stencil programs.

The fused horizontal diffusion + vertical advection program (and its
unfused, adjoint and batched-timestep forms) runs as hand-written HIP
kernels for gfx950 inside ``libstencil.so``, behind the C ABI of
``include/stencil.h``.  This package is the thin Python binding of that
library (``binding``), an autograd wrapper (``autograd``), the build driver
(``build``) and the seeded input generators (``inputs``).

The binding is imported lazily so that ``inputs`` can be used without torch.
"""

_BINDING_NAMES = {
    "Field", "FieldDesc", "Config", "Program", "ProgramSpec", "Subdomain", "StencilError", "config", "lib",
    "stencil_hdiff", "stencil_vadv", "stencil_hdiff_vadv", "stencil_hdiff_vadv_adjoint",
    "stencil_program_run", "stencil_probe_copy", "stencil_last_error", "stencil_abi_version",
    "stencil_shutdown", "EXPORTS", "LIB_PATH",
}


def __getattr__(name):
    if name in _BINDING_NAMES:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
