"""Plain CPU oracle for the halftoning hot path -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package; the product library never imports it.
"""
