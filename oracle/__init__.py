"""FP64 CPU oracle for the line-by-line cross-section hot path (TEST INFRASTRUCTURE).

This package is test infrastructure.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library never
calls into it and shares no code with it.

It is a plain, slow, obviously-correct transcription of the definitions in the
ExoCross paper (Yurchenko, Al-Refaie & Tennyson 2018): every function cites the
section and equation it follows.  Floating point is IEEE double throughout; the
Faddeeva function is SciPy's ``wofz`` (a library special function), sums over
states use ``math.fsum`` (correctly rounded).
"""
from .constants import *  # noqa: F401,F403
from .xsec import *  # noqa: F401,F403
from .vvoigt import *  # noqa: F401,F403
from .binned import *  # noqa: F401,F403
from .threshold import *  # noqa: F401,F403
from .emission import *  # noqa: F401,F403
from .nonlte import *  # noqa: F401,F403
