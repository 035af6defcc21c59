"""Plain FP64 CPU oracle of the HSGN/SWE time step (test infrastructure only)."""
