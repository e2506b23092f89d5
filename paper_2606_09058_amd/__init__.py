"""MI355X-native generalized Kohn-Sham eigensolver and density build (gfx950 HIP)."""
