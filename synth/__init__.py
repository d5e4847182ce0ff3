"""Seeded synthetic inputs (scenes, cameras) shared by the oracle tests, the
GPU tests and the benchmark.  Contains no rendering arithmetic."""
from .scenes import (Camera, Gaussians, Scene, Surfels, workload, perturbed_copy,
                     permute_gaussians, permute_surfels, pinhole, ring_camera, subset,
                     empty_gaussians, empty_surfels, SH_K, SH_DEGREE)
