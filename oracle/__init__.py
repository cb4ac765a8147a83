"""Plain CPU oracle for pixel-level CKKS (test infrastructure only)."""
