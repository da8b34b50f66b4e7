"""FP64 CPU oracle of the two-component Shan-Chen D3Q19 step (test infrastructure only)."""
