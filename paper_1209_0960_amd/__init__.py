"""MI355X-native non-smoothed aggregation AMG-preconditioned CG (Blatt, Ippisch, Bastian).

The HIP library is loaded lazily on first use of the solver API, so that the
workload generator in :mod:`paper_1209_0960_amd.problems` can be imported on a
machine without a GPU.
"""
