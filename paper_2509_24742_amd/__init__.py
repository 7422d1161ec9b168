"""SRBE constant-potential step on MI355X (gfx950)."""
