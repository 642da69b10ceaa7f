"""FP64 CPU oracle of the CTU-PPM + HLLC hydro step.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; the product path never imports it.
"""
