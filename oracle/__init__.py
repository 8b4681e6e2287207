"""FP64 CPU oracle.  Test infrastructure: only the tests, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does."""
