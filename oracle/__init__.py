"""CPU oracle for the GIFT search stage (test infrastructure only).

This package is a plain, slow reference written from the paper.  It is not
part of the product: only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import it.  It shares no code with the HIP path.
"""
from .gift_oracle import *  # noqa: F401,F403
