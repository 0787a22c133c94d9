"""CPU FP64 oracle for the multi-stage preconditioned GMRES path.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` import this package.  The product library
(``paper_1912_04385_amd``) shares no code with it and never calls it.

Parity unpinned: the learned-interpolation forward pass is pinned only by
properties (zero correction reproduces the classical weights; a finite
difference check of its gradient), not by anything the paper prints.
"""
from .core import *  # noqa: F401,F403
