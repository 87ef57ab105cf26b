"""FP64 reference implementation of the simulator.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it to check and time the GPU library; the library and
its binding never import it.
"""
