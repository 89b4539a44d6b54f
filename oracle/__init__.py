"""CPU oracle for the three-bead swimmer step (test infrastructure only).

A plain, slow NumPy implementation, in float64 (or complex128 for the
complex-step tangent), of the coupled lattice-Boltzmann / rigid-body step of
Pickl et al., "All good things come in threes - Three beads learn to swim with
lattice Boltzmann and a rigid body solver" (arXiv:1108.0786): Alg. 2 of
Sec. 2.3, with the LBGK collision of Sec. 2.1 (Eqs. lbgk, collide, streaming),
halfway bounce-back (Eq. lbm:bounce_back), the moving-object bounce-back and
momentum-exchange force of Sec. 2.3 (Eq. hydroF), the spring-damper forces of
Sec. 2.2 (Eqs. spring_i, damp_i, osci_i/j) and the driving protocol of
Sec. 3.3 (Eqs. FB1-FB3).

It is test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the
GPU library in ``paper_1108_0786_amd``; both take their inputs from
``workloads``.

Every function cites the passage it follows.  Readings of points the paper
leaves open are listed in the module docstrings where they are used.
"""
from .d3q19 import E, W, OPP, Q
from .sim import OracleSim, run_case

__all__ = ["E", "W", "OPP", "Q", "OracleSim", "run_case"]
