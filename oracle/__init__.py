"""CPU oracle for the 3D multiscale DRT / DJT (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library neither imports nor links
it, and the two share no code.
"""
from .oracle import *  # noqa: F401,F403
from .inverse import *  # noqa: F401,F403
from .net import *  # noqa: F401,F403
from .planes import *  # noqa: F401,F403
