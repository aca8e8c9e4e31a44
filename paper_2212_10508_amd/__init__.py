"""MI355X-native batched SNAP + Langevin fine propagator for adaptive parareal."""
