"""CPU FP64 oracle of the lattice sweep. TEST INFRASTRUCTURE ONLY.

Used by tests/, by the entry point's smoke check and by the benchmark's CPU-baseline
leg. The library and its Python binding never import it, and it imports nothing from
them.
"""
