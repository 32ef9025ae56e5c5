"""Exact (delta13, delta12, delta23)-temporal triangle counting on MI355X (gfx950).

The work happens in libdottt.so (HIP kernels behind the C ABI of include/dottt.h); this package
only marshals arguments to it (see dottt.py).  Build the library with
paper_2106_02762_amd.build.build().
"""
from .dottt import *  # noqa: F401,F403
from .dottt import DtError, library, make_query  # noqa: F401
