"""Test infrastructure: the plain FP64 CPU reference of the method.

Only tests, the package smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it."""
