"""FP64 reference oracle (test infrastructure only; see oracle.py)."""
