"""FP64 CPU oracle for the 3D-RISM solver -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, deliberately unoptimised restatement of the
method of arXiv 2403.01039 (sections "Theory", "Numerical procedure",
"Convergence acceleration") in float64 numpy.  It exists to check the HIP
library.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path (the C-ABI library and its Python
binding) never imports, links or calls anything here, and shares no code with
it: the oracle has its own FFT (``oracle.fft``), its own potential, closures,
MDIIS and free-energy sums (``oracle.rism3d``), and its own 1D RISM / DRISM
solvent solver (``oracle.rism1d``) that produces the solvent susceptibility
tables both sides read.

Pinning (what checks the oracle against something other than itself) lives in
``tests/test_oracle_*.py``; every function here names the passage it follows.
"""
