"""Seeded synthetic inputs (test and benchmark infrastructure)."""
