"""MI355X-native multilevel BDDC (Sistek, Mandel, Sousedik, Burda, "Parallel
implementation of Multilevel BDDC").

The numerical work lives in the HIP library libmlbddc.so (C ABI in
include/mlbddc.h); this package is its Python binding.
"""

from ._lib import MlbddcError, load  # noqa: F401
from .solver import BDDCSolve, Problem, Solver, element_load, element_matrix  # noqa: F401
