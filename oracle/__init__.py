"""FP64 CPU oracle for tree-structured coupled OT (test infrastructure only).

Only the test suite, the smoke entry point and the CPU-baseline leg of the
benchmark may import this package.  It never depends on the HIP path.
"""
from .tree_ot import TreeOracle, logsumexp, validate_tree

__all__ = ["TreeOracle", "logsumexp", "validate_tree"]
