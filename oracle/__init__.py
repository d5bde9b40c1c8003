"""Plain, slow FP64 CPU oracle for the DG + multi-rate AB3 + imaging hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import anything here; the product path never does.
It shares no code with the HIP library (paper_1506_00907_amd/csrc); the only
common input is the seeded generator module paper_1506_00907_amd.inputs.
"""
