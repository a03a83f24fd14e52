"""MI355X-native CoRdE Cosserat-rod stepper: HIP kernels for gfx950 behind a C ABI.

The compiled library ``libcorde_rod.so`` (sources in ``csrc/``, declarations in
``include/rod.h``) does all the stepping; ``paper_2509_04277_amd.rod`` is a thin ctypes binding
with the same entry-point names.  ``workloads`` holds the seeded synthetic inputs.
"""
__all__ = ["rod", "workloads"]
