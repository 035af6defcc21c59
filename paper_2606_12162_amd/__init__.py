"""MI355X-native HSGN/SWE time step (placeholder, filled below)."""
