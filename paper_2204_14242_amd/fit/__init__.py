"""Fitting the capacity-miss model's hit-rate functions to volumes measured
on the GPU (Sec. 4.5): measurement kernels (star_probe.hip), the counter
collection driver (measure.py) and the least-squares fit (fit.py)."""
