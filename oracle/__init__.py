"""FP64 CPU oracle of the phase-field lattice Boltzmann step (test infrastructure only)."""
