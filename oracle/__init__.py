"""FP64 CPU oracle of the spherical 2D-surfel rasterizer (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The product path never does.
"""
from .oracle import *  # noqa: F401,F403
from .adam import adam_step  # noqa: F401
from .loss import loss_l1_normal  # noqa: F401
from .gn import huber, pose_gn, pose_jacobian  # noqa: F401
from . import photo  # noqa: F401
from .photo import photo_gn  # noqa: F401
from . import mapping  # noqa: F401
