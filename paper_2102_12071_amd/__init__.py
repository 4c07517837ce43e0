"""mgcnn: geometric multigrid with a learned per-point smoother on AMD MI355X.

The compute path is the HIP library ``libmgcnn.so`` behind the C ABI in
``include/mgcnn.h``; ``mgcnn`` is its Python binding (argument marshalling
only).  Build with ``python -m paper_2102_12071_amd.build``.
"""
from . import mgcnn  # noqa: F401
from .mgcnn import (Context, MGError, Net, Options, TrainOptions, galerkin, load_library,  # noqa: F401
                    stencil_cellavg5, stencil_q1_rotated)
