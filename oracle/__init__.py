"""Float64 CPU oracle for the DMALA MIMO detector.

TEST INFRASTRUCTURE: a plain, slow, independent implementation of the method,
used only by tests/, __graft_entry__.smoke() and the CPU-baseline leg of
bench.py.  It shares no code with the HIP library and the library never
imports it.  Modules:

* philox -- Philox4x32-10 (Salmon et al., SC'11) and the random-word layout;
* dmala  -- system model, proposal, Algorithm 1, estimators, Algorithm 2;
* exact  -- enumeration over A^N: posterior, exact LLRs/marginals, MAP,
            transition matrix, convergence rate, TV distance;
* learned -- learned proposal (network, features), its mixture with the plain
            kernel, exact mixture kernels, training loss, gradients and Adam.
"""
from . import philox, dmala, exact, learned  # noqa: F401
