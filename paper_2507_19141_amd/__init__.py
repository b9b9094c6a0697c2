"""MI355X-native DASH 4D hash deformation path (HIP library + thin Python binding)."""
