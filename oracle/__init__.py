"""CPU oracle of the implicit electron / electric-potential step (test infrastructure only)."""
