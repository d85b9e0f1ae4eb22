"""Seeded synthetic radar frames shared by the tests and the benchmark."""
