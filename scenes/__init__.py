"""Seeded synthetic street-corridor inputs.

This package only *draws* inputs: Gaussian attributes, instance trajectories,
camera rigs, render targets and the initial temporal-visibility state.  It holds
none of the rendering method's arithmetic (no projection, culling, sorting,
compositing or visibility update), so both the CPU oracle and the GPU path can
consume the same inputs without sharing any code of the method.
"""

from .corridor import (  # noqa: F401
    SEED_BASE,
    Scene,
    Views,
    default_params,
    make_config,
    make_scaleup,
    micro_scene,
    targets,
)
