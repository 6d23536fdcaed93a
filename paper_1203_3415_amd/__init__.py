"""MI355X (gfx950) exact directed motif census for k = 3, 4, 5 (and 6).

Thin Python binding over the C ABI of ``libmotif.so`` (declared in
``include/motif.h``).  Every step of the census runs in the library's HIP
kernels; this package only marshals arguments.  Importing it does not load
the library; the first call does, and raises if the library was not built.
"""
from .binding import (  # noqa: F401
    MotifError,
    NUM_CLASSES,
    lib,
    lib_path,
    census,
    census6,
    class6_codes,
    class6_multiplicities,
    NUM_CLASSES6,
    census_async,
    census_undirected,
    num_undirected_classes,
    undirected_class_code,
    class_undirected,
    NUM_UNDIRECTED_CLASSES,
    census_batch,
    census_multi,
    census_batch_loop,
    BatchPlan,
    null_randomize,
    null_model,
    num_classes,
    class_code,
    class_multiplicity,
    class_of_code,
    read_network,
    get_tuning,
    set_tuning,
    autotune,
    tune_cache_save,
    tune_cache_load,
    profile_enable,
    profile_read,
    to_device,
    Server,
    request_footprint,
)
from .nullmodel import zscores  # noqa: F401,E402
