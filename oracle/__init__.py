"""FP64 CPU oracle of the guided filter and the Fast Guided Filter.

Test infrastructure only (tests, the smoke check, the benchmark's CPU
baseline); the GPU library never imports it.
"""
