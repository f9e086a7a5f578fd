"""CPU oracle for the GST likelihood path -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does.
"""
from .binding import (  # noqa: F401
    build, probs, probs_extended, loglik, vjp, tv_distance, predict, OracleError, library_path,
)
from . import params  # noqa: F401  (parameterizations of the fit)
from . import fit  # noqa: F401  (LGST, MLGST, gauge optimization)
from . import metrics  # noqa: F401  (post-fit metrics)
