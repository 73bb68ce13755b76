"""FP64 CPU oracle of the 4D Gaussian rendering routine (test infrastructure only)."""
