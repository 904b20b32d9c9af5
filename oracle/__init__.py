"""CPU oracle for the Paillier hot path -- test infrastructure only.

Importable by ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py``; never by the product library.
"""
from .paillier import *  # noqa: F401,F403
