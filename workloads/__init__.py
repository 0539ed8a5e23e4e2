"""Seeded synthetic inputs (circuits, occupation patterns) shared by the oracle's tests and the GPU path."""
