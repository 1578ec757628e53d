"""Interval branch-and-bound global minimisation on AMD MI355X (gfx950)."""
