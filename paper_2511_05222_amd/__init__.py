"""MI355X-native VMC force hot path (Jastrow-Slater determinant in a GTO basis).

Importing the package loads nothing; the HIP library is loaded on first use by
:mod:`paper_2511_05222_amd.vmc` and fails loudly if it has not been built.
"""
__all__ = ["inputs", "vmc"]
