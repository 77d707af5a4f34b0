"""FP64 CPU oracle of the VIF approximation -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. The product path (the HIP library and its binding) never
calls it and shares no code with it.
"""
