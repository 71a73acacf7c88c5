"""Seeded synthetic workloads (shapes, parameters, masks, inputs) shared by the
oracle tests and the GPU path's tests and benchmark.  No arithmetic of the
method lives here."""
from .configs import EvoConfig, PRESETS, SUBOPS, TEMPLATE_SUBOPS, get, param_spec  # noqa: F401
from .inputs import (SEED, make_inputs, make_masks, make_params, make_template_inputs,  # noqa: F401
                     make_template_params, round_inputs, to_storage)
