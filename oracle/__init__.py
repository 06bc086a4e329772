"""CPU FP64 oracle for the blob reaction-diffusion solves.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU baseline import it. ``exact`` holds the plain definitions and exact
(FFT + dense) solves; ``iterative`` binds the plain C multigrid/Krylov
implementation in ``blob_oracle.c``. Neither shares code with the HIP path.
"""
