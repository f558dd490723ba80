"""FP64 CPU oracle of the EIS-inversion grid search (test infrastructure only)."""
