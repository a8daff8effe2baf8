"""MI355X-native boundary-layer-preconditioned FGMRES (arXiv 2108.13468).

Importing the package loads nothing; `paper_2108_13468_amd.blp` is the binding
of the HIP library (it raises if the library is not built).
"""
