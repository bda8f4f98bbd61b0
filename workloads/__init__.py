"""Seeded synthetic inputs shared, as data, by the oracle and the GPU path."""
