"""libpolydg: MI355X (gfx950) HIP implementation of the modal-time-stepping DGSEM residual on
mixed hexahedral / prismatic / pyramidal / tetrahedral meshes, with Hilbert-curve ordering
and cost-weighted work queues.  The C ABI is include/pdg.h; `binding.PolyDG` wraps it."""


def __getattr__(name):
    if name in ("PolyDG", "load_library", "PdgError"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
