"""Double-precision CPU oracle of the particle-in-cell step (test infrastructure only)."""
