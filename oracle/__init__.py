"""CPU FP64 oracle of the GMG Poisson V-cycle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the product path never imports it.
"""
