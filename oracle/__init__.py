"""CPU oracle of the diffuse-interface step -- test infrastructure only.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never does.
"""
