"""MI355X (gfx950) implementation of the data-parallel hot path of MG-GLAM
(Ruan et al., arXiv:2110.00328): CIC density assignment, the nonlinear FAS
multigrid solve of the f(R) / symmetron / coupled-quintessence scalar field,
the fifth force, and their adjoints, behind the C ABI in include/mggpu.h.

``paper_2110_00328_amd.api`` holds the torch-facing wrappers; importing this
package does not import torch.
"""
from . import _lib  # noqa: F401
