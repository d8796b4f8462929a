"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the simulation method: it only draws the
random initial noise and names the workload parameter sets. Both the CPU
oracle and the GPU library consume what it produces.
"""
from .noise import splitmix64_uniforms, gaussian_noise, initial_omega
from .presets import PRESETS, base_params, preset, replica_manifest

__all__ = ["splitmix64_uniforms", "gaussian_noise", "initial_omega",
           "PRESETS", "base_params", "preset", "replica_manifest"]
