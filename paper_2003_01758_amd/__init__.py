"""MI355X-native hot path of the Parallel Constrained Bernstein Algorithm (PCBA).

Submodules are imported lazily: `instances` (seeded workloads) never loads the
HIP library; `pcba` (the C-ABI binding) fails loudly if the library is missing.
"""
