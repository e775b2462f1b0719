"""Python binding of the MI355X Langevin-XY library (placeholder, filled in below)."""
