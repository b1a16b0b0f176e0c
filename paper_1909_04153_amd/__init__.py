"""MI355X-native adaptive-AB3 extended-Boussinesq time stepper (arXiv 1909.04153).

The solver itself lives in the HIP library ``csrc/`` built into
``libbq.so``; ``bq`` is its ctypes binding and ``scenarios`` the seeded input
generators.
"""
