"""MI355X-native nodal DG reverse-time migration (pressure-velocity system, multi-rate AB3, characteristic imaging).

Importing the package is cheap: the HIP library binding lives in
`paper_1506_00907_amd.dgrtm` and is loaded on first use.
"""
__version__ = "0.1.0"
