"""FP64 CPU oracle (test infrastructure only; see nmf_oracle)."""
