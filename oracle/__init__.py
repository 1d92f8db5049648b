"""FP64 CPU oracle for the DGSM hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference written directly from the paper's equations.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path (``paper_2601_01660_amd``)
and imports nothing from it.

Modules
-------
``dgsm``  build and query of the transmittance atlas (Sec. 3.2-3.3, Eqs. 1-5)
``sh``    real SH basis, probe evaluation and radiance transfer (Sec. 3.4-3.5)
``mlp``   the learned per-light transmittance field (forward, backward, Adam)
"""
from . import dgsm, sh, mlp  # noqa: F401
