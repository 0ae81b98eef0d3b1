"""FP64 CPU oracle for Block CUR.  Test infrastructure only: imported by the
tests, the entry script's smoke check and the benchmark's CPU-baseline leg,
never by the product path."""
from . import bcur_oracle  # noqa: F401
