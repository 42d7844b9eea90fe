"""Seeded synthetic inputs shared by the CPU oracle and the GPU path."""
from .jacobian import System, generate, redraw_values  # noqa: F401
