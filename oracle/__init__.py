"""CPU FP64 oracle (test infrastructure only; see bltt_oracle)."""
