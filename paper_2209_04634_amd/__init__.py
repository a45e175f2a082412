"""MI355X-native event simulator: frame pairs in, time-ordered (x, y, t, polarity) events out.

The compute path lives in the HIP library built from `csrc/`; `sim` is its thin ctypes binding.
Importing this package loads nothing; `paper_2209_04634_amd.sim` loads the library on first use.
"""
