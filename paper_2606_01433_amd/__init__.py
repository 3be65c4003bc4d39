"""MI355X-native monolithic multilevel GDSW overlapping Schwarz for Q2-P1disc Stokes systems."""
