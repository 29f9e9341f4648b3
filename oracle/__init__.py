"""FP64 CPU oracle for the radiative-transfer lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the HIP library or its binding.
It shares no code with the HIP path; the only common module is
``workloads`` (seeded inputs, no arithmetic of the method).
"""
