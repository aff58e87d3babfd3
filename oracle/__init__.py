"""FP64 CPU oracle of the diffuse-solid lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU baseline of
the benchmark use it to check the GPU library; the GPU library never does.
"""
