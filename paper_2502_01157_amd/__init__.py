"""MI355X (gfx950) Voronoi ray walk: the forward and backward hot path of
Radiant Foam (differentiable ray tracing through a Voronoi tessellation).

The compute lives in librf.so (HIP, C ABI in include/radfoam.h); this package
is the thin Python binding. Importing it loads the library and fails if it is
missing.
"""

from . import _lib
from ._lib import RfError  # noqa: F401

_lib.lib()  # fail loudly when the HIP library has not been built

from .ops import (  # noqa: E402,F401
    DEFAULT_EPS,
    DEFAULT_LOG_CAPACITY,
    DEFAULT_MAX_STEPS,
    AdamState,
    PackedScene,
    Quantiles,
    RadFoamRender,
    Surface,
    WalkLog,
    adam_step,
    densify_scores,
    gather_rows,
    insert_sites,
    keep_index,
    locate,
    prune_mask,
    quantile_forward,
    raygen,
    render,
    render_backward,
    render_forward,
    render_trace,
    sample_cells,
    train_schedule,
)

__version__ = "0.1.0"
