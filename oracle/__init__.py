"""CPU oracle (test infrastructure only; see binary_lbm.py)."""
