"""CPU reference (test infrastructure only; see oracle.py)."""
