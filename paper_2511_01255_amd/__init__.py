"""MI355X-native HWSDA hot path (quasi-phase-matching crystal design)."""
