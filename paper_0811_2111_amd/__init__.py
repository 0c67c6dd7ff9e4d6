"""Checkerboard Metropolis sweeps of the 2-d XY model on MI355X (gfx950).

The compute path is the HIP library ``libxyhip.so`` (C ABI: include/xy.h);
``paper_0811_2111_amd.xy`` is its Python binding.
"""
