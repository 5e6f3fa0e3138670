"""MI355X twofold arithmetic (placeholder; the binding is added with the HIP library)."""
