"""CPU oracle (test infrastructure only; see qed_oracle's module docstring)."""
