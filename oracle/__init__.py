"""CPU oracle of the IWFPM Hamiltonian and eigenproblem (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package; the product path never imports it.
"""

from .iwfpm_oracle import *  # noqa: F401,F403
