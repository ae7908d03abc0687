"""ORACLE -- test infrastructure only.

Plain, slow, obviously correct CPU FP64 implementations of what the GPU path
computes: the direct convolution sum with singularity subtraction (C, threaded)
and a treecode taking the paper's Algorithm 3 steps in order (numpy), plus the
closed forms that pin them. Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import anything here; the product library never does.
"""
