"""MI355X-native Aggregate Risk Analysis (ARA): a C-ABI library of gfx950
HIP kernels (``libara.so``, see ``include/ara.h``) and its Python binding."""
from .ara import Ara, AraError, Server, evaluations, lib  # noqa: F401
