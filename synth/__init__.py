"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package holds only input generation: images, random weights and the
weight-blob byte format. It holds none of the compression method's
arithmetic (no model evaluation, no CDFs, no coder), so that neither
implementation can lean on the other through it.
"""
from .images import (  # noqa: F401
    smooth_field_image,
    workload_images,
    workload_shapes,
    WORKLOADS,
    training_pool,
    training_crops,
)
from .weights import (  # noqa: F401
    MODEL_DIMS,
    param_shapes,
    param_count,
    init_params,
    write_blob,
    fnv1a64,
    model_blob,
    delta_params,
)
