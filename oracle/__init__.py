"""FP64 CPU oracle for the superiorized conjugate gradient hot path.

TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py may import this package. The product path (the
HIP library and its binding in paper_1709_04912_amd) never imports it, and the
two share no code.

Operators live in plain C (oracle_ops.c, built to liboracle.so with gcc); the
algorithm drivers (CG, S-CG, S-CG-CD, S-PCG, the K-restarted variants and the
perturbation procedure) are plain numpy in algorithms.py, each following the
paper's algorithm of the same name step by step.
"""
from .ops import Geometry, build, lib_path  # noqa: F401
from . import algorithms  # noqa: F401
