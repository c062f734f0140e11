"""RaBitQ query-phase estimation for MI355X (gfx950): C-ABI library + Python binding."""
from . import rabitq  # noqa: F401
from .rabitq import Index, RbqError  # noqa: F401
