"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

Holds no arithmetic of the segmentation method: only images, codebooks and parameters.
"""
from .workloads import (Workload, make_c0, make_c1, make_c2, make_c3, make_c3_image, make_c4,
                        make_config, make_denoise, make_small, random_data, random_image)

__all__ = ["Workload", "make_c0", "make_c1", "make_c2", "make_c3", "make_c3_image", "make_c4",
           "make_config", "make_denoise", "make_small", "random_data", "random_image"]
