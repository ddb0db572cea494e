"""CPU FP64 oracle for the QMC sector-integration path.  TEST INFRASTRUCTURE.

Plain, slow, obviously correct reimplementation of what the GPU path
computes, written from the paper.  Only tests, the smoke check and the CPU
baseline of the benchmark may import anything from this package; the
product path never does.
"""
