"""MI355X-native recursive module-coupling eigensolver (HIP/gfx950)."""
