"""CPU FP64 oracle (test infrastructure only; see txe_oracle)."""
