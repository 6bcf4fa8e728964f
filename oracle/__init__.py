"""Plain CPU FP64 oracle of the crack-length-controlled phase-field FFT solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it exists so that `tests/`, the smoke check and the CPU
baseline leg of the benchmark can compare the HIP implementation against a
slow, obviously correct restatement of the paper (Aranda & Segurado, "A
crack-length control technique for phase field fracture in FFT
homogenization").  It shares no code with the HIP path; the only common
dependency is the `synth` package of seeded input generators.

Modules
-------
fourier   frequencies, Willot-rotated projection, spectral Laplacian (Sec. 3.1)
pointlaw  spectral strain split, degraded stress and tangent, history (Sec. 2.1, 2.3, 3.2)
system    residual F and tangent action dF of the crack-length system (Sec. 3.2)
krylov    plain BiCGSTAB and CG
newton    Newton loop, increments and bootstrap (Algorithm 2)
brute     dense finite-difference-Jacobian Newton for tiny grids
appendix  Fourier crack-functional amplification factor (Appendix A.1)

Every function is pinned by `tests/test_oracle_*.py` against closed forms,
invariants, brute force or values printed in the paper.
"""

from . import fourier, pointlaw, system, krylov, newton, brute, appendix  # noqa: F401
