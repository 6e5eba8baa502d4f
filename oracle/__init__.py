"""FP64 CPU oracle of the Directional TSDF hot path (test infrastructure only)."""
