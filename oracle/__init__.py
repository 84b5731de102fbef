"""FP64 CPU oracle of the IMPM substep -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package.  The product library never links, loads or calls it.
"""
