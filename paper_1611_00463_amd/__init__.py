"""Load-balanced sample sort for AMD MI355X (gfx950)."""
