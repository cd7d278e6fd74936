"""MI355X incremental GPU snapshot: Python binding of libcrum.

The C ABI (``include/crum.h``) is the product boundary; this package only
marshals arguments to it (``_lib``) and offers a small convenience layer
(:mod:`.api`) that owns pinned status/image buffers as torch tensors.
"""
from ._lib import *  # noqa: F401,F403
from ._lib import lib, read_status, region_table, Plan, Server, Writer, read_request_statuses  # noqa: F401,E501
from ._lib import Lazy, ImageError, Tracker  # noqa: F401
from .build import build  # noqa: F401
