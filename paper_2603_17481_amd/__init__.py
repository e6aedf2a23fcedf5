"""MI355X-native coupled lattice Boltzmann / conservative Allen-Cahn step with
near-contact repulsion (arXiv:2603.17481)."""
