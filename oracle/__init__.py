"""CPU oracle for wedge sampling (test infrastructure only; see oracle.py)."""
