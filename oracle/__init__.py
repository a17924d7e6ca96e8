"""Plain FP64 CPU oracle of weighted quadrature (WQ) on unstructured bicubic splines.

TEST INFRASTRUCTURE ONLY. Imported by tests/, by the package smoke check and by the
benchmark's CPU-baseline leg; the GPU library never imports, links or calls it, and it
shares no code with the GPU library. It is slow and written to be read against the
paper (Sections 2-5), step by step.
"""
from .wq import *  # noqa: F401,F403
from . import heat  # noqa: F401,E402
