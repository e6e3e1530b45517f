"""FP64 CPU oracle of the gain-dissipative method (test infrastructure only)."""
