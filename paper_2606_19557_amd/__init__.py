"""MI355X-native NEP training hot path (descriptors, E/F/virial, loss, analytic
parameter gradient, Adam) behind the libnep C ABI. See ``nep.py``."""

from .nep import (  # noqa: F401
    AdamConfig,
    Batch,
    Model,
    NEPFunction,
    Neighbors,
    NepError,
    Plan,
    Targets,
    Zbl,
    nep_adam_step,
    nep_autotune,
    nep_backward,
    nep_build_neighbors,
    nep_descriptor_scale,
    nep_descriptors,
    nep_forward,
    nep_gather_batch,
    nep_loss_and_grad,
    nep_param_count,
    nep_profile_enable,
    nep_profile_read,
    nep_workspace_size,
    nep_zbl_add,
    workspace,
)
