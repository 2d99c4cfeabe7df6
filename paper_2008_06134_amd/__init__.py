"""Slice-based ray-casting volume illumination on MI355X (gfx950).

The HIP library ``libvi.so`` (built from ``csrc/``) holds both passes of the
method -- the light-space attenuation build and the eye-space ray march --
behind the C-ABI declared in ``include/vi.h``.  ``vi`` is its thin ctypes
binding.  Importing this package loads nothing; ``paper_2008_06134_amd.vi``
loads the library on first use and raises if it is missing.
"""
