"""FP64 CPU reference of the particle step (test infrastructure only)."""
