"""CPU oracle for the Barnes-Hut potential path -- test infrastructure only.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library never does, and this package never
imports the product library.
"""
from .oracle import OracleTree, build_oracle, oracle_library_path  # noqa: F401
