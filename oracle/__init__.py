"""CPU FP64 oracle for the Zakharov/HOS wave step.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library under ``paper_2608_25203_amd/``; the two meet only through the seeded
input generators in ``paper_2608_25203_amd/inputs.py``, which hold none of
the method's arithmetic.

Modules
-------
hos      grid, DFT backends, dealiased product, Craig-Sulem/HOS DtN series,
         Bernoulli term, Zakharov RHS, RK4 + state filter, Hamiltonian.
laplace  dense direct Laplace solve of the Dirichlet-Neumann problem, the
         independent check of the series (no series arithmetic inside).
cnn      plain im2col CNN (forward, backward, Adam) for the learned closure.
"""
