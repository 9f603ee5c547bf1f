"""CPU oracle for warm-start APSP -- test infrastructure only (see oracle.py)."""
