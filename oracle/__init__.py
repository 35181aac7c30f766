"""CPU oracle for the EBCC hot path (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product (the GPU library and its Python binding)
never imports, links or calls it.
"""
