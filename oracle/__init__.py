"""FP64 CPU oracle (test infrastructure only; see radar_oracle.py)."""
