"""MI355X-native interior-point discarding for 2D convex hulls (placeholder)."""
