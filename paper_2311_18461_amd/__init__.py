"""MI355X-native space-time fast-diagonalisation solver for the Schrodinger equation.

The compute path is the C ABI library ``libstfd.so`` (include/stfd.h) with its
ctypes binding in ``paper_2311_18461_amd.stfd``, which only marshals
arguments.  ``paper_2311_18461_amd.inputs`` holds seeded problem data and can
be imported without the library.
"""
