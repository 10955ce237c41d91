"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package holds only input recipes: procedural triangle scenes, start
states and action sequences drawn from ``numpy.random.default_rng(seed)``,
cast to float32 once.  It contains none of the simulator's arithmetic (no
dynamics, no ray casting); both the oracle and the device path receive the
same arrays from here and compute independently.
"""
from .params import default_params, device_params, PARAM_FIELDS
from . import scenes, agents

__all__ = ["default_params", "device_params", "PARAM_FIELDS", "scenes", "agents"]
