"""Seeded synthetic inputs (Voronoi meshes, direction sets, coefficient fields) shared by
the oracle, the tests and the benchmark.  Holds no part of the sweep's arithmetic."""
