"""MI355X-native multidimensional included and excluded sums (HIP for gfx950)."""
