"""CPU FP64 oracle (test infrastructure only: tests, the smoke entry and the
benchmark's CPU-baseline leg use it; the product path never does)."""
