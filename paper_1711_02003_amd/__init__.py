"""Regularized colour-gradient lattice Boltzmann on AMD MI355X (gfx950)."""
