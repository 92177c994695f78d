"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds input generation only (microstructures, material tables,
load paths). It contains none of the solver's arithmetic, so both the CPU
oracle and the HIP path can draw identical inputs from it without sharing
any of the method's code.
"""
from .microstructure import inclusion_microstructure, laminate_microstructure
from .workloads import (MATRIX_DAMAGE, MATRIX_TENSILE, INCLUSION_ELASTIC, Workload, workload,
                        uniaxial_load_path)

__all__ = ["inclusion_microstructure", "laminate_microstructure",
           "MATRIX_DAMAGE", "MATRIX_TENSILE", "INCLUSION_ELASTIC", "Workload", "workload",
           "uniaxial_load_path"]
