"""FP64 CPU oracle of the TVLBM step -- test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library does not.
"""
