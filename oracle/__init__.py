"""FP64 CPU oracle for the SBI wave solver -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct numpy implementation of what the GPU path
computes, written from the paper (Wang, "An Enhanced Spectral Boundary Integral
Method for Modeling Highly Nonlinear Water Waves in Variable Depth"):

* Sec. 2.2, Eq. (prognostic) and its integrating-factor form: the time step
  (fixed-step RK4, and the adaptive embedded fifth/fourth-order pair);
* Sec. 2.4 (successive approximations) with Appendix C, Eqs. (v2)-(v7): the
  surface vertical velocity V;
* Sec. 3.1, Eq. (energy): the total energy diagnostic;
* Sec. 3.3, Eq. (filter): the optional low-pass filter;
* Sec. 3.2: the numerical wave tank's pneumatic wavemaker and damping
  pressure (Eq. (pd));
* ``fenton``: exact steady (Stokes) waves in deep water and finite depth by the
  stream-function method, the reference of the accuracy studies of Sec. 4 and
  Sec. 5;
* ``warmstart``: the learned warm start of the W iteration (features, network
  forward and backward, Adam), defined in that module's header.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does; it
shares no code, tables or constants with this package.
"""
from .sbi_oracle import (  # noqa: F401
    Grid,
    Solver,
    SolveInfo,
    lawson_rk54,
    w_sa_appc,
)
from . import dft  # noqa: F401
from . import fenton  # noqa: F401
from . import warmstart  # noqa: F401
from . import history_seed  # noqa: F401
