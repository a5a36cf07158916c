"""FP64 CPU oracle of the collocation BEM of arXiv 2312.12787 (ctypes binding).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the
product package ``paper_2312_12787_amd``; the two see the same seeded inputs
(``workloads``) and nothing else.
"""
from .oracle import *  # noqa: F401,F403
