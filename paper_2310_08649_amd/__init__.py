"""Time-vectorized backward-Euler integration of batched stiff ODEs on MI355X (gfx950)."""
