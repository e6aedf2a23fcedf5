"""CPU FP64 oracle of the coupled lattice step -- test infrastructure only."""
