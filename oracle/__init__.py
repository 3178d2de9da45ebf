"""FP64 CPU oracle (test infrastructure only; never called by the product path)."""
