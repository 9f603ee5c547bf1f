"""The paper's own warm-start procedures (Algorithms 5, 6, 7 and 11) on one
CPU thread, with the cold starts they are compared with, to re-run the
paper's warm/cold experiments on known hardware.  Benchmark and test
infrastructure: nothing on the GPU path uses it, and it shares no code with
the HIP library or with the oracle."""
