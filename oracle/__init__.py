"""FP64 CPU oracle for the fused D3Q19 MRT pseudopotential + D3Q7 MRT thermal
lattice Boltzmann step of Li, Yu & Luo (arXiv:2201.06039).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import anything from here; the
HIP library never does, and nothing here imports the HIP library.

Modules:
  build    -- compiles lbm_oracle.c into liboracle.so with gcc (OpenMP, -O2,
              no fast-math).
  sim      -- ctypes wrapper of the C oracle (whole-grid passes, FP64).
  thermo   -- Peng-Robinson EOS, Maxwell equal-area coexistence and the
              closed-form PR fugacity used to pin it.
"""
