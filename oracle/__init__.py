"""FP64 CPU oracle of the Dirac sweep -- test infrastructure only (see oracle.py)."""
