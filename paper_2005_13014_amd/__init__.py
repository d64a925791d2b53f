"""Placeholder; the binding is added with the HIP library."""
