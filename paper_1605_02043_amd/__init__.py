"""Edge-partitioned kernels for MI355X (gfx950).

Python face of libepk (see include/epk.h): partition a data-affinity graph,
pack it along the task order and run the partition-ordered FLUX5 / SpMV
kernels.  Importing fails loudly if libepk.so has not been built.
"""

from ._lib import EpkError, lib  # noqa: F401  (raises ImportError if the library is missing)
from .plan import Plan, partition, permute_rows  # noqa: F401

__all__ = ["Plan", "partition", "permute_rows", "EpkError", "lib"]
