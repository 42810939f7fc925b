"""MI355X-native lattice sweep of the LPC3D mesoscopic model (hop + precess + moments).

Importing the package loads nothing native; `paper_2603_22553_amd.lattice` loads the HIP
C-ABI library `liblpc.so` and raises if it has not been built.
"""
