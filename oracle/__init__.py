"""FP64 CPU reference of the PIC cycle -- test infrastructure only (see oracle.c)."""
