"""FP64 CPU oracle of the FITrig hot path (test infrastructure only)."""
