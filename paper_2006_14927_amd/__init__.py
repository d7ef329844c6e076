"""MI355X-native Cherenkov photon-bunch generation and atmospheric propagation.

Importing the package loads nothing native; `paper_2006_14927_amd.ckv`
loads the HIP library on first use and raises if it is missing.
"""
