"""Seeded synthetic inputs for the power-Doppler reconstruction path.

This package is shared by the GPU path's tests/bench and by the CPU oracle.
It generates *inputs only*: acquisition parameters (probe, transmits, voxel
grid, slow-time sampling) and scatterer scenes (positions per frame and
reflectivities), plus seeded random RF / IQ arrays used as stage inputs.
It holds none of the reconstruction arithmetic (no delays, no pulse model,
no demodulation, no beamforming, no clutter filtering).
"""
from .configs import Acq, SceneSpec, CONFIGS, MOTION_SWEEP, augmented_motion_config, get_config, motion_sweep_configs  # noqa: F401
from .scene import Scene, make_scene, rigid_motion, tissue_displacement  # noqa: F401
from .random_inputs import random_rf, random_casorati, lcf_init_weights, batch_indices  # noqa: F401
