"""CPU oracle for the Gross-Pitaevskii split step (arXiv:2003.03590).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 numpy
restatement of the paper's method, written independently of the HIP library:
it shares no code, header, table or helper with ``paper_2003_03590_amd`` and
never imports it.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path must never
route through it.

Modules
  fft      -- dense DFT (definition) and a plain mixed-radix FFT
  gp       -- Strang split step, mass/energy, hydrodynamic energy split,
              shell spectra, density structure function, parameter rules
  adjoint  -- adjoint of the split step, spectral loss and its gradient

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
invariants, brute force or values printed in the paper.
"""
from . import fft, gp, adjoint  # noqa: F401
