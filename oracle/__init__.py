"""FP64 CPU oracle for the SRD-MPCD time step (Howard, Panagiotopoulos and
Nikoubashman, "Efficient mesoscale hydrodynamics: multiparticle collision
dynamics with massively parallel GPU acceleration", arXiv:1801.10187).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it. The GPU library never
calls it, links it or falls back to it, and it shares no code with the GPU
path: it has its own Philox, its own binning, sums, draws and rotation.

Modules
-------
philox    Philox4x32-10 counter-based generator (Salmon et al., SC'11) and the
          word -> uniform mapping; vectorised numpy and a scalar form.
srd       One SRD step in plain FP64 numpy (sec. 2 eq. 1-3, sec. 3.4-3.6,
          Alg. 1): stream, grid shift, bin, cell sums, rotation axis,
          Maxwell-Boltzmann cell thermostat, rotation.
fp32form  Emulation of the FP32 cell-relative storage form: every single
          precision operation done in numpy float32, the collision in FP64
          (sec. 4.1 mixed-precision model).
brute     Pure-Python loops with exact rational sums for boxes of at most a
          few cells; pins the vectorised code.

Parity status: every function here is pinned by the CPU tests (known-answer
vectors, closed forms, library routines, invariants, brute force); none is
"parity unpinned".
"""
