"""CPU FP64 oracle for the demag-extrapolated explicit LLG method.

This package is TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(the HIP library and its Python binding) never imports, calls or links it, and
shares no code with it: the only common module is ``workloads`` (seeded input
generators, no arithmetic of the method).

Everything is plain NumPy/SciPy in float64, written for a reader who checks it
against the paper (Lepadatu, "Speeding up explicit numerical evaluation methods
for micromagnetic simulations using demagnetizing field polynomial
extrapolation", arXiv:2107.06729):

* ``newell``     demagnetizing tensor of Sec. II / Eq. (2) (formulas of ref. [24])
* ``demag``      Eq. (2): direct O(N^2) sum and zero-padded FFT convolution
* ``fields``     H_eff terms named under Eq. (1) and the LLG right-hand side
* ``tableaux``   Butcher tableaux of the methods listed in Sec. II
* ``integrate``  Eq. (3)-(4) stepping, Eq. (5) controller, Eq. (6) extrapolation
* ``metrics``    Eq. (7) error and averages

Parity status of every function is stated in its module docstring; functions
with no independent pin say "parity unpinned".
"""

from . import newell, demag, fields, tableaux, integrate, metrics  # noqa: F401
