"""MI355X (gfx950) randomized minimal-norm solver (Tygert, arXiv 0905.4745).

The method runs in the HIP library libminnorm.so (C ABI in include/minnorm.h);
this package only marshals torch tensors into that ABI.  Importing the API
requires the built library: there is no CPU fallback.
"""

from ._lib import LIB_PATH, EXPORTS  # noqa: F401


def __getattr__(name):
    # lazy: `import paper_0905_4745_amd` works without a GPU; the entry points
    # load the library (and fail loudly if it is missing) on first use
    if name in ("srft_sketch", "build_preconditioner", "minnorm_solve", "minnorm_solve_batched",
                "SolveOptions", "MinnormError", "workspace_bytes"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
