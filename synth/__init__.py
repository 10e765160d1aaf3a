"""Seeded synthetic input events (shared input generator; no method arithmetic)."""
