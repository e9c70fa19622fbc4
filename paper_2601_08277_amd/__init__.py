"""MI355X-native particle-in-cell current deposition (MatrixPIC, arXiv 2601.08277)."""
