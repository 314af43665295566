"""CPU FP64 oracle of the hybrid SP-Shakhov / DSMC particle update (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The product path never does.
"""
from .oracle import Oracle, build_oracle, lib  # noqa: F401
