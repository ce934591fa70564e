"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *draws* inputs: coarse (macro) meshes of a channel with an
obstacle, random solver states and random network weights.  It contains none
of the method's arithmetic (no refinement, no quadrature, no solver, no
network evaluation), so the oracle and the HIP path can both consume it
without sharing any code of the method.
"""
from .channel import (MacroMesh, channel_obstacle, channel_obstacles, rectangle,
                      random_state, gru_weights, training_channel, WORKLOADS)

__all__ = ["MacroMesh", "channel_obstacle", "channel_obstacles", "rectangle",
           "random_state", "gru_weights", "training_channel", "WORKLOADS"]
