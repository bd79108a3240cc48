"""sFMM on MI355X (placeholder; the binding is added with the library)."""
