"""MI355X-native CSPH-TVD shallow-water solver (arXiv 1705.00614 hot path)."""
