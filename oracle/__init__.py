"""FP64 CPU oracle of the per-patch MOL hydro update (test infrastructure only)."""
