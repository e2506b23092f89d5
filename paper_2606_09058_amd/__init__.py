"""MI355X-native (gfx950) generalized Kohn-Sham eigensolver and density build.

The solve runs in the HIP library ``libks.so`` (C-ABI in include/ks.h); the
Python binding ``paper_2606_09058_amd.ks`` only marshals tensors into it.
``paper_2606_09058_amd.inputs`` draws the seeded synthetic workloads.
"""
