"""MI355X-native D2Q9 Shan-Chen lattice Boltzmann with the EWOD electric force.

The package holds the HIP library (``csrc/``), its ctypes binding (``lbm``) and
the seeded synthetic input generators (``inputs``).  Importing the package does
not load the native library; ``paper_0708_4182_amd.lbm`` does that on first use
and raises if it has not been built.
"""

__all__ = ["inputs", "lbm"]
