"""Null-collision Monte Carlo path tracing through hierarchical majorant grids
(Villefranque et al., JAMES 2019) on MI355X: HIP kernels behind a C ABI
(include/nctrace.h), with a thin Python binding (`api`)."""
